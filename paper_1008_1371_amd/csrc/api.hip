// C ABI of libhsvd (include/hsvd.h) and the host driver of the sweep loop.
//
// The driver follows the structure of the paper's host routine (Alg. 4.1):
// set-up and Precompute_Data, Sort_Diagonal, then sweeps of parallel steps,
// each sweep ending with the convergence check and another sort.  The only
// host synchronisation inside a solve is one small copy of the control block
// per sweep, which decides whether another sweep is launched.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "internal.h"

struct hsvd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    void *aux = nullptr;                     // buffers of a solve with jsig in any order, autotuner input
    size_t aux_bytes = 0;
    hsvd::Ctl *host_ctl = nullptr;           // pinned
    hsvd::PersistCtl *host_pctl = nullptr;   // pinned, in the same allocation
    std::vector<hipEvent_t> events;          // reusable timing events
    hipStream_t cap = nullptr;               // non-blocking stream for graph capture (default priority)
    hipEvent_t join = nullptr;               // orders the capture stream with the caller's stream
    struct Tune {
        int valid = 0, algo = 0, wg = 0;
    } tune[16];                              // autotuner choice per size bucket (log2 of n, rounded up)
    // threads per workgroup of the persistent batched kernel, by the bucket of
    // the largest order in the launch ((0, 64], (64, 128], (128, 192],
    // (192, 256]); 0 = the default
    int persist_threads[4] = {0, 0, 0, 0};
    // sweep schedule of batch_mode 2 per precision (FP64, mixed): 0 = one
    // persistent launch, 1 = launches grouped by order; -1 = not tuned
    int batch_sched[2] = {-1, -1};
};

// Fixed device scratch of hsvd_solve_noalloc: the workspace of one solve,
// for callers that cannot allocate device memory.  Each device holds its own
// copy for the life of the process.  Host code never names the array in a
// device context: its device address comes from hipGetSymbolAddress, taken
// once per device in hsvd_init (with that device current) and kept in
// g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[HSVD_NOALLOC_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device `device` (looked up on
// the first call for that device).  Null if the lookup failed.
void *scratch_address(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[device] = ptr;
    }
    return g_scratch_ptr[device];
}

}  // namespace

namespace {

int size_bucket(int n)
{
    int b = 0;
    while ((1 << b) < n && b < 15) ++b;
    return b;
}

void tune_load(hsvd_ctx *ctx)
{
    const char *path = getenv("HSVD_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char buf[4096];
    const size_t len = fread(buf, 1, sizeof(buf) - 1, f);
    fclose(f);
    buf[len] = 0;
    // entries written by tune_save: {"bucket": B, "algo": A, "wg": W}
    for (const char *q = strstr(buf, "\"bucket\""); q; q = strstr(q + 1, "\"bucket\"")) {
        int b = -1, a = 0, w = 0;
        if (sscanf(q, "\"bucket\": %d, \"algo\": %d, \"wg\": %d", &b, &a, &w) == 3 && b >= 0 && b < 16 &&
            (a == HSVD_PAIRWISE || a == HSVD_BLOCK) && w >= 0) {
            ctx->tune[b].valid = 1;
            ctx->tune[b].algo = a;
            ctx->tune[b].wg = w;
        }
    }
    // {"batched_bucket": B, "threads": T}
    for (const char *q = strstr(buf, "\"batched_bucket\""); q; q = strstr(q + 1, "\"batched_bucket\"")) {
        int b = -1, t = 0;
        if (sscanf(q, "\"batched_bucket\": %d, \"threads\": %d", &b, &t) == 2 && b >= 0 && b < 4 &&
            (t == 256 || t == 512 || t == 1024))
            ctx->persist_threads[b] = t;
    }
    // {"batched_schedule": P, "mode": M}
    for (const char *q = strstr(buf, "\"batched_schedule\""); q; q = strstr(q + 1, "\"batched_schedule\"")) {
        int pr = -1, m = -1;
        if (sscanf(q, "\"batched_schedule\": %d, \"mode\": %d", &pr, &m) == 2 && (pr == 0 || pr == 1) &&
            (m == 0 || m == 1))
            ctx->batch_sched[pr] = m;
    }
}

void tune_save(const hsvd_ctx *ctx)
{
    const char *path = getenv("HSVD_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "w");
    if (!f) return;
    fprintf(f, "{\"library\": \"%s\", \"entries\": [", "hsvd-gfx950");
    bool first = true;
    for (int b = 0; b < 16; ++b) {
        if (!ctx->tune[b].valid) continue;
        fprintf(f, "%s\n  {\"bucket\": %d, \"algo\": %d, \"wg\": %d}", first ? "" : ",", b, ctx->tune[b].algo,
                ctx->tune[b].wg);
        first = false;
    }
    for (int b = 0; b < 4; ++b) {
        if (!ctx->persist_threads[b]) continue;
        fprintf(f, "%s\n  {\"batched_bucket\": %d, \"threads\": %d}", first ? "" : ",", b, ctx->persist_threads[b]);
        first = false;
    }
    for (int pr = 0; pr < 2; ++pr) {
        if (ctx->batch_sched[pr] < 0) continue;
        fprintf(f, "%s\n  {\"batched_schedule\": %d, \"mode\": %d}", first ? "" : ",", pr, ctx->batch_sched[pr]);
        first = false;
    }
    fprintf(f, "\n]}\n");
    fclose(f);
}

}  // namespace

namespace hsvd {

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

Layout make_layout(int n, int r, int ldg, bool want_v, int pairs, int splits, int b2, bool mixed)
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
    L.off_rtmp = take(sizeof(int) * 2 * (size_t)r);  // sort: moved rho, then ranks
    L.off_S = take(sizeof(int4) * slots);
    L.off_C = take(sizeof(int) * slots);
    L.off_nrot = take(sizeof(unsigned int) * slots);
    L.off_nskip = take(sizeof(unsigned int) * slots);
    L.off_nact = take(sizeof(unsigned int) * slots);
    L.off_ntc = take(sizeof(unsigned int) * slots);
    L.off_maxt = take(sizeof(double) * slots);
    L.off_ctl = take(sizeof(Ctl));
    L.off_ver = take(sizeof(unsigned int) * r);
    L.off_pctl = take(sizeof(PersistCtl));
    const size_t bb = (size_t)b2 * b2;
    L.off_P = take(sizeof(double) * (size_t)pairs * splits * bb);
    // W and the touched-column masks are double-buffered by step parity: the
    // V update of a step runs inside the next step's inner launch
    L.off_W = take(sizeof(double) * (size_t)pairs * bb * 2);
    L.off_active = take(sizeof(unsigned long long) * (size_t)pairs * 2);
    L.off_S2 = take(sizeof(int4) * 2 * (size_t)pairs);
    L.mixed = mixed;
    const size_t mat = (size_t)ldg * r;
    L.off_G32 = take(mixed ? sizeof(float) * mat : 0);
    L.off_V32 = take(mixed ? sizeof(float) * mat : 0);
    L.off_P32 = take(mixed ? sizeof(float) * (size_t)pairs * splits * bb : 0);
    L.off_W32 = take(mixed ? sizeof(float) * (size_t)pairs * bb * 2 : 0);
    L.off_T1 = take(mixed ? sizeof(double) * mat : 0);
    L.off_T2 = take(mixed ? sizeof(double) * mat : 0);
    const bool wide = b2 == 2 * kWideB;
    L.wide = wide;
    L.off_G2 = take(wide ? sizeof(double) * mat : 0);
    L.off_V2 = take(wide && want_v ? sizeof(double) * mat : 0);
    L.off_blk = take(wide ? sizeof(int2) * (size_t)pairs : 0);
    L.off_pl = take(wide ? sizeof(int) * (size_t)r : 0);
    L.off_rho2 = take(wide ? sizeof(int) * (size_t)r : 0);
    L.off_wact = take(wide ? sizeof(int) * (size_t)pairs : 0);
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
    w.ntc = reinterpret_cast<unsigned int *>(b + L.off_ntc);
    w.maxt = reinterpret_cast<double *>(b + L.off_maxt);
    w.ctl = reinterpret_cast<Ctl *>(b + L.off_ctl);
    w.ver = reinterpret_cast<unsigned int *>(b + L.off_ver);
    w.pctl = reinterpret_cast<PersistCtl *>(b + L.off_pctl);
    if (L.pairs > 0) {
        w.P = reinterpret_cast<double *>(b + L.off_P);
        w.W = reinterpret_cast<double *>(b + L.off_W);
        w.active = reinterpret_cast<unsigned long long *>(b + L.off_active);
        w.S2 = reinterpret_cast<int4 *>(b + L.off_S2);
    }
    if (L.mixed) {
        w.G32 = reinterpret_cast<float *>(b + L.off_G32);
        w.V32 = L.off_P32 > L.off_V32 ? reinterpret_cast<float *>(b + L.off_V32) : nullptr;
        w.P32 = reinterpret_cast<float *>(b + L.off_P32);
        w.W32 = reinterpret_cast<float *>(b + L.off_W32);
        w.T1 = L.off_T2 > L.off_T1 ? reinterpret_cast<double *>(b + L.off_T1) : nullptr;
        w.T2 = L.bytes > L.off_T2 ? reinterpret_cast<double *>(b + L.off_T2) : nullptr;
    }
    if (L.wide) {
        w.G2 = reinterpret_cast<double *>(b + L.off_G2);
        w.V2 = L.off_blk > L.off_V2 ? reinterpret_cast<double *>(b + L.off_V2) : nullptr;
        w.blk = reinterpret_cast<int2 *>(b + L.off_blk);
        w.pl = reinterpret_cast<int *>(b + L.off_pl);
        w.rho2 = reinterpret_cast<int *>(b + L.off_rho2);
        w.wact = reinterpret_cast<int *>(b + L.off_wact);
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
    prm->graph = 1;
    prm->inner_sweeps = 0;
    prm->reorth_accept = 0.0;
    prm->batch_mode = 2;
    prm->persistent = 0;
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
    const size_t pctl_at = align_up(sizeof(Ctl), 64);
    if (hipHostMalloc(&h, pctl_at + sizeof(PersistCtl), hipHostMallocDefault) != hipSuccess) {
        delete ctx;
        return HSVD_E_DEVICE;
    }
    ctx->host_ctl = static_cast<Ctl *>(h);
    ctx->host_pctl = reinterpret_cast<PersistCtl *>(static_cast<char *>(h) + pctl_at);
    if (!scratch_address(device)) {
        hipHostFree(h);
        delete ctx;
        return HSVD_E_DEVICE;
    }
    tune_load(ctx);
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
    if (ctx->aux) hipFree(ctx->aux);
    if (ctx->host_ctl) hipHostFree(ctx->host_ctl);
    if (ctx->cap) hipStreamDestroy(ctx->cap);
    if (ctx->join) hipEventDestroy(ctx->join);
    delete ctx;
    return HSVD_OK;
}

}  // extern "C"

namespace {

// Per-sweep diagnostics on stderr when HSVD_SWEEP_LOG is set (non-empty, not "0").
bool sweep_log_enabled()
{
    static const bool on = [] {
        const char *v = getenv("HSVD_SWEEP_LOG");
        return v && *v && strcmp(v, "0") != 0;
    }();
    return on;
}

// Outcome of one sweep, read back from the control block.
struct SweepResult {
    int code;
    double maxt;
    bool rank;
};

// Kernel timing of the block sweeps: an event pair around every kernel of
// every step would itself cost several microseconds per launch, so the
// first step of a sweep (its own inner kernel) and every kTimeEvery-th step
// after it are timed, and the other steps of the sweep are counted at the
// mean of its timed ones.
constexpr int kTimeEvery = 8;

// Capture of one sweep's launches on the context's capture stream (default
// priority, non-blocking) and its replay.  begin() joins the capture stream
// to the caller's stream and starts capturing; end() instantiates.  The
// destructor frees the graph and joins the caller's stream back to the
// capture stream, on every exit path.
struct SweepGraph {
    hsvd_ctx *ctx;
    hipStream_t st;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool used = false;
    SweepGraph(hsvd_ctx *c, hipStream_t s) : ctx(c), st(s) {}
    hipError_t begin(hipStream_t &q)
    {
        hipError_t e;
        if (!ctx->cap && (e = hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking)) != hipSuccess) return e;
        if (!ctx->join && (e = hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming)) != hipSuccess) return e;
        q = ctx->cap;
        used = true;
        if ((e = hipEventRecord(ctx->join, st)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(q, ctx->join, 0)) != hipSuccess) return e;
        return hipStreamBeginCapture(q, hipStreamCaptureModeThreadLocal);
    }
    hipError_t end(hipStream_t q)
    {
        hipError_t e = hipStreamEndCapture(q, &graph);
        if (e != hipSuccess) return e;
        return hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    }
    void abort(hipStream_t q)
    {
        hipGraph_t g = nullptr;
        if (hipStreamEndCapture(q, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
    }
    ~SweepGraph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (used && hipEventRecord(ctx->join, ctx->cap) == hipSuccess) (void)hipStreamWaitEvent(st, ctx->join, 0);
    }
};

// Runs block sweeps of storage type T until `done(sweep_result)` says so or
// max_sweeps is reached.  Kernel times go to kms[kbase + 0..2] (Gram, inner,
// update), the number of timed launches to ktimed.  Returns HSVD_OK,
// HSVD_E_RANK or HSVD_E_DEVICE; *finished tells whether `done` accepted a
// sweep.
template <typename T, typename Done>
hsvd_status block_sweeps(hsvd_ctx *ctx, const Workspace &w, BlockArgsT<T> &ba, const T *Gcur, int pairs,
                         int steps_per_sweep, int max_sweeps, bool sort, int r, int p, int ldg, long long &gstep,
                         int kbase, double *kms, long long *klaunch, long long *ktimed, int &sweeps,
                         long long &steps, SweepResult &last, bool &finished, bool timing, Done done)
{
    hipStream_t st = ctx->stream;
    // timing: event pairs around sampled launches (the events exist; see
    // ensure_events); otherwise no event is recorded
    hipEvent_t *ev = timing ? ctx->events.data() : nullptr;
    hipEvent_t *evv = timing ? ev + 4 + 4 * steps_per_sweep : nullptr;  // around the V update of a sweep's last step
    finished = false;
    // W and the masks alternate between two buffers by step parity.  With V
    // accumulated by the block-oriented method, the V half of a step's update
    // runs as extra workgroups of the next step's inner launch (on the CUs the
    // inner solves leave idle; the next Gram needs G alone), and the last
    // step's in an update launch of its own at the end of the sweep.
    const size_t wstride = (size_t)pairs * (2 * block_width()) * (2 * block_width());
    T *const Wb = ba.W;
    unsigned long long *const Ab = ba.active;
    const bool fuse = ba.V != nullptr && ba.inner_sweeps == 0 && ba.nprob <= 1;
    int cus = 0;
    if (fuse && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess)
        return HSVD_E_DEVICE;
    ba.vrows = fuse ? v_update_role_rows(pairs, ldg, cus, sizeof(T) == 8) : 0;
    const int vwgs = fuse ? v_update_role_wgs(pairs, ldg, ba.vrows) : 0;
    for (int sw = 0; sw < max_sweeps; ++sw) {
        for (int k = 0; k < steps_per_sweep; ++k, ++gstep) {
            const int par = (int)(gstep & 1);
            ba.step = k;
            ba.S_in = w.S2 + par * pairs;
            ba.S_out = w.S2 + (par ^ 1) * pairs;
            ba.W = Wb + par * wstride;
            ba.active = Ab + par * pairs;
            ba.vprev_wgs = 0;
            if (fuse && k > 0) {
                ba.vprev_wgs = vwgs;
                ba.W_prev = Wb + (par ^ 1) * wstride;
                ba.active_prev = Ab + (par ^ 1) * pairs;
                ba.S_prev = w.S2 + (par ^ 1) * pairs;  // the previous step's S_in: rewritten by this step's update
                ba.step_prev = k - 1;
            }
            hipEvent_t *e = timing ? ev + 4 + 4 * k : nullptr;
            const bool tm = timing && k % kTimeEvery == 0;
            if (tm) HSVD_TRY(hipEventRecord(e[0], st));
            HSVD_TRY(launch_block_gram<T>(st, ba));
            if (tm) HSVD_TRY(hipEventRecord(e[1], st));
            HSVD_TRY(launch_block_inner<T>(st, ba));
            if (tm) HSVD_TRY(hipEventRecord(e[2], st));
            HSVD_TRY(launch_block_update<T>(st, ba, fuse ? UPD_G : UPD_BOTH));
            if (tm) HSVD_TRY(hipEventRecord(e[3], st));
        }
        if (fuse) {
            const int par = (int)((gstep - 1) & 1);
            BlockArgsT<T> lv = ba;
            lv.step = steps_per_sweep - 1;
            lv.S_in = w.S2 + par * pairs;
            lv.W = Wb + par * wstride;
            lv.active = Ab + par * pairs;
            lv.vprev_wgs = 0;
            if (timing) HSVD_TRY(hipEventRecord(evv[0], st));
            HSVD_TRY(launch_block_update<T>(st, lv, UPD_V));
            if (timing) HSVD_TRY(hipEventRecord(evv[1], st));
        }
        for (int q = 0; q < 3; ++q) klaunch[kbase + q] += steps_per_sweep;
        // the kept diagonal: fresh column norms of the updated columns
        HSVD_TRY(launch_colnorm_pos<T>(st, Gcur, ldg, w.rho, w.d, r));
        steps += steps_per_sweep;
        if (sort) HSVD_TRY(launch_sort(st, w.d, w.rho, w.dtmp, w.rtmp, r, p));
        HSVD_TRY(launch_sweep_reduce(st, w, pairs));
        HSVD_TRY(hipMemcpyAsync(ctx->host_ctl, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
        HSVD_TRY(hipStreamSynchronize(st));
        if (timing) {
            double first[3] = {0.0, 0.0, 0.0}, rest[3] = {0.0, 0.0, 0.0};
            int nrest = 0;
            for (int k = 0; k < steps_per_sweep; k += kTimeEvery) {
                hipEvent_t *e = ev + 4 + 4 * k;
                for (int q = 0; q < 3; ++q) {
                    float ms = 0.f;
                    HSVD_TRY(hipEventElapsedTime(&ms, e[q], e[q + 1]));
                    (k == 0 ? first : rest)[q] += ms;
                }
                if (k > 0) ++nrest;
            }
            const double scale = nrest > 0 ? (double)(steps_per_sweep - 1) / nrest : 0.0;
            for (int q = 0; q < 3; ++q) {
                kms[kbase + q] += first[q] + rest[q] * scale;
                ktimed[kbase + q] += 1 + nrest;
            }
            if (fuse) {
                float ms = 0.f;
                HSVD_TRY(hipEventElapsedTime(&ms, evv[0], evv[1]));
                kms[kbase + 2] += ms;
                ktimed[kbase + 2] += 1;
            }
        }
        if (fuse) klaunch[kbase + 2] += 1;
        ++sweeps;
        last.code = ctx->host_ctl->code;
        last.maxt = ctx->host_ctl->maxt;
        last.rank = ctx->host_ctl->rank != 0;
        if (sweep_log_enabled())
            fprintf(stderr, "hsvd sweep %d (%s): max|t| %.3e code %d rotations %llu skips %llu\n", sweeps,
                    sizeof(T) == 4 ? "fp32" : "fp64", last.maxt, last.code,
                    (unsigned long long)ctx->host_ctl->rot, (unsigned long long)ctx->host_ctl->skip);
        if (last.rank) {
            ba.W = Wb;
            ba.active = Ab;
            ba.vprev_wgs = 0;
            return HSVD_E_RANK;
        }
        if (done(last)) {
            finished = true;
            break;
        }
    }
    ba.W = Wb;
    ba.active = Ab;
    ba.vprev_wgs = 0;
    return HSVD_OK;
}

// FP64 sweeps of the wide block path (b = 64): working copies in position
// order (gathered from the input order after the first sort, moved after
// every later sort), Gram and update on the block-pair form of the FP64 MFMA
// GEMM, inner rotations in wide_inner_kernel.  On return, out_G / out_V /
// out_rho hold G and V in the input's column order and rho, as finalize reads
// them.  Kernel times as block_sweeps (first step of each sweep and every
// kTimeEvery-th step after it timed).
hsvd_status wide_sweeps(hsvd_ctx *ctx, const Workspace &w, int r, int p, int ldg, int nb, int splits, int ordering,
                        bool want_v, bool sort, double tol, double tthresh, int inner_sweeps, int max_sweeps,
                        bool timing, double *kms, long long *klaunch, long long *ktimed, int &sweeps,
                        long long &steps, SweepResult &last, bool &finished, double *&out_G, double *&out_V,
                        int *&out_rho)
{
    hipStream_t st = ctx->stream;
    const int pairs = nb / 2, b2 = 2 * kWideB;
    const int steps_per_sweep = ordering == HSVD_ORD_MODMOD ? nb : nb - 1;
    double *Gc = w.G2, *Gn = w.G, *Vc = want_v ? w.V2 : nullptr, *Vn = want_v ? w.V : nullptr;
    int *rc = w.rho, *rn = w.rho2;
    // to position order: column q <- input column rho[q]
    HSVD_TRY(launch_wide_move(st, w.G, Gc, ldg, r, w.rho, false, nullptr, nullptr));
    if (want_v) HSVD_TRY(launch_wide_move(st, w.V, Vc, ldg, r, w.rho, false, nullptr, nullptr));
    GemmArgs gram;  // partial[pair][split] = G_P(rows of split)^T G_P(rows of split)
    gram.B = nullptr;
    gram.C = w.P;
    gram.M = gram.N = b2;
    gram.K = ldg / splits;
    gram.ldb = gram.lda = ldg;
    gram.ldc = b2;
    gram.sc = (long long)b2 * b2;
    gram.blk = w.blk;
    gram.bw = kWideB;
    gram.map = 1 | 2;
    gram.ksplit = splits;
    GemmArgs upd;  // [G_P | V_P] <- [G_P | V_P] W, in place, pairs with a rotation only
    upd.M = ldg;
    upd.N = upd.K = b2;
    upd.lda = upd.ldc = ldg;
    upd.ldb = b2;
    upd.B = w.W;
    upd.sb = (long long)b2 * b2;
    upd.blk = w.blk;
    upd.bw = kWideB;
    upd.map = 1 | 4;
    upd.flag = w.wact;
    upd.want = 1;
    WideArgs wa;
    wa.partial = w.P;
    wa.splits = splits;
    wa.W = w.W;
    wa.blk = w.blk;
    wa.p = p;
    wa.tol = tol;
    wa.tthresh = tthresh;
    wa.inner_sweeps = inner_sweeps;
    wa.active = w.wact;
    wa.C = w.C;
    wa.nrot = w.nrot;
    wa.nskip = w.nskip;
    wa.nact = w.nact;
    wa.ntc = w.ntc;
    wa.maxt = w.maxt;
    wa.ctl = w.ctl;
    hipEvent_t *ev = timing ? ctx->events.data() : nullptr;
    finished = false;
    long long gstep = 0;
    for (int sw = 0; sw < max_sweeps; ++sw) {
        double first[3] = {0.0, 0.0, 0.0}, rest[3] = {0.0, 0.0, 0.0};
        int nrest = 0;
        for (int k = 0; k < steps_per_sweep; ++k, ++gstep) {
            const int par = (int)(gstep & 1);
            const bool tm = timing && k % kTimeEvery == 0;
            hipEvent_t *e = tm ? ev + 4 + 4 * k : nullptr;
            HSVD_TRY(launch_wide_blk(st, ordering, nb, k, w.S2 + par * pairs, w.S2 + (par ^ 1) * pairs, w.blk));
            if (tm) HSVD_TRY(hipEventRecord(e[0], st));
            gram.A = gram.B = Gc;
            HSVD_TRY(launch_gemm(st, gram, pairs * splits, true, false, true));
            if (tm) HSVD_TRY(hipEventRecord(e[1], st));
            wa.first = k == 0 ? 1 : 0;
            HSVD_TRY(launch_wide_inner(st, wa, pairs));
            if (tm) HSVD_TRY(hipEventRecord(e[2], st));
            upd.A = Gc;
            upd.C = Gc;
            HSVD_TRY(launch_gemm(st, upd, pairs, false, false, false));
            if (want_v) {
                upd.A = Vc;
                upd.C = Vc;
                HSVD_TRY(launch_gemm(st, upd, pairs, false, false, false));
            }
            if (tm) HSVD_TRY(hipEventRecord(e[3], st));
        }
        for (int q = 0; q < 3; ++q) klaunch[HSVD_K_BLOCK_GRAM + q] += steps_per_sweep;
        steps += steps_per_sweep;
        // the kept diagonal (fresh norms, by position), the sort and the column moves
        HSVD_TRY(launch_wide_iota(st, w.pl, r));
        HSVD_TRY(launch_colnorm_pos<double>(st, Gc, ldg, w.pl, w.d, r));
        if (sort) {
            HSVD_TRY(launch_sort(st, w.d, w.pl, w.dtmp, w.rtmp, r, p));  // pl: the old position now at q
            HSVD_TRY(launch_wide_move(st, Gc, Gn, ldg, r, w.pl, false, rc, rn));
            if (want_v) HSVD_TRY(launch_wide_move(st, Vc, Vn, ldg, r, w.pl, false, nullptr, nullptr));
            std::swap(Gc, Gn);
            std::swap(Vc, Vn);
            std::swap(rc, rn);
        }
        HSVD_TRY(launch_sweep_reduce(st, w, pairs));
        HSVD_TRY(hipMemcpyAsync(ctx->host_ctl, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
        HSVD_TRY(hipStreamSynchronize(st));
        if (timing) {
            for (int k = 0; k < steps_per_sweep; k += kTimeEvery) {
                hipEvent_t *e = ev + 4 + 4 * k;
                for (int q = 0; q < 3; ++q) {
                    float ms = 0.f;
                    HSVD_TRY(hipEventElapsedTime(&ms, e[q], e[q + 1]));
                    (k == 0 ? first : rest)[q] += ms;
                }
                if (k > 0) ++nrest;
            }
            const double scale = nrest > 0 ? (double)(steps_per_sweep - 1) / nrest : 0.0;
            for (int q = 0; q < 3; ++q) {
                kms[HSVD_K_BLOCK_GRAM + q] += first[q] + rest[q] * scale;
                ktimed[HSVD_K_BLOCK_GRAM + q] += 1 + nrest;
            }
        }
        ++sweeps;
        last.code = ctx->host_ctl->code;
        last.maxt = ctx->host_ctl->maxt;
        last.rank = ctx->host_ctl->rank != 0;
        if (last.rank) break;
        if ((last.code & 2) == 0) {
            finished = true;
            break;
        }
    }
    // back to the input's column order for finalize: column rho[q] <- column q
    HSVD_TRY(launch_wide_move(st, Gc, Gn, ldg, r, rc, true, nullptr, nullptr));
    if (want_v) HSVD_TRY(launch_wide_move(st, Vc, Vn, ldg, r, rc, true, nullptr, nullptr));
    out_G = Gn;
    out_V = Vn;
    out_rho = rc;
    return last.rank ? HSVD_E_RANK : HSVD_OK;
}

// Newton-Schulz J-re-orthogonalisation of X (in w.V, FP64, promoted from the
// FP32 sweeps), X <- X (3I - J X^T J X) / 2, followed by G <- G X.  The
// products run on the library's FP64 MFMA kernels (X^T J X as a symmetric
// product with J applied to the rows of the second operand as it is loaded).
// Uses w.T1, w.T2.  iters: corrections applied; resid: max |J X^T J X - I| of
// the final X.  With gx = false G is left alone.
hsvd_status reorthogonalise(hsvd_ctx *ctx, const Workspace &w, int n, int r, int p, int ldg, int &iters,
                            double &resid, bool gx = true)
{
    hipStream_t st = ctx->stream;
    iters = 0;
    resid = 1.0;
    double prev = 2.0;
    // residual at the level of the rounding of the products themselves: the
    // n real columns (the bordering columns are exact unit vectors and add
    // no rounding)
    const double floor_ = 16.0 * n * 0x1p-53;
    GemmArgs sy;  // T2 = X^T J X
    sy.A = w.V;
    sy.B = w.V;
    sy.C = w.T2;
    sy.M = sy.N = sy.K = r;
    sy.lda = sy.ldb = sy.ldc = ldg;
    sy.p = p;
    GemmArgs xt = sy;  // T1 = X T2
    xt.B = w.T2;
    xt.C = w.T1;
    for (int it = 0; it <= 6; ++it) {
        HSVD_TRY(launch_gemm(st, sy, 1, true, true, true));
        ctx->host_ctl->nsres = 0.0;
        HSVD_TRY(hipMemcpyAsync(&w.ctl->nsres, &ctx->host_ctl->nsres, sizeof(double), hipMemcpyHostToDevice, st));
        HSVD_TRY(launch_ns_form(st, w.T2, p, ldg, r, w.ctl));  // T2 = (3I - J X^T J X) / 2
        HSVD_TRY(hipMemcpyAsync(&ctx->host_ctl->nsres, &w.ctl->nsres, sizeof(double), hipMemcpyDeviceToHost, st));
        HSVD_TRY(hipStreamSynchronize(st));
        resid = ctx->host_ctl->nsres;
        // stop once X is J-orthogonal to working accuracy (residual at the
        // rounding floor, or no longer falling quadratically; or after six
        // corrections) -- that last correction is not applied; the caller
        // judges the final residual
        if (it == 6 || !(resid < 1.0) || resid <= floor_ || (iters > 0 && resid > 0.25 * prev)) break;
        HSVD_TRY(launch_gemm(st, xt, 1, false, false, false));
        HSVD_TRY(launch_copy(st, w.T1, w.V, ldg, r));
        ++iters;
        prev = resid;
    }
    if (gx) {
        GemmArgs g1 = sy;  // T1 = G X
        g1.A = w.G;
        g1.B = w.V;
        g1.C = w.T1;
        HSVD_TRY(launch_gemm(st, g1, 1, false, false, false));
        HSVD_TRY(launch_copy(st, w.T1, w.G, ldg, r));
    }
    return HSVD_OK;
}

// Largest accepted final residual of the J-re-orthogonalisation.
double reorth_accept_bound(const hsvd_params &prm, int n)
{
    return prm.reorth_accept > 0.0 ? prm.reorth_accept : 16384.0 * n * 0x1p-53;
}

}  // namespace

namespace {

// Where a solve's workspace comes from, and what it may create.
struct SolveMode {
    void *ws = nullptr;   // nullptr: the context's workspace (allocated or grown on demand)
    size_t ws_cap = 0;    // bytes available at ws
    bool timing = true;   // HIP events around the solve and sampled kernels (events are created on demand)
    bool graphs = true;   // prm.graph honoured (a captured graph is created per solve)
    hsvd_status too_big = HSVD_E_NOMEM;  // returned when ws is set and the solve needs more than ws_cap
};

// hsvd_solve for J = diag(I_p, -I_{n-p}) (columns in canonical order).
hsvd_status solve_canonical(hsvd_ctx *ctx, const double *G, int lda, int n, int p, const hsvd_params &prm,
                            double *sigma, double *U, int ldu, double *V, int ldv, double *lambda, int *perm,
                            hsvd_info *info, const SolveMode &mode)
{
    if (info) memset(info, 0, sizeof(*info));
    if (!ctx || !G || !sigma) return HSVD_E_INVAL;
    if (n < 1 || p < 0 || p > n || lda < n) return HSVD_E_INVAL;
    if (U && ldu < n) return HSVD_E_INVAL;
    if (V && ldv < n) return HSVD_E_INVAL;
    if (prm.ordering != HSVD_ORD_MODMOD && prm.ordering != HSVD_ORD_ROUNDROBIN) return HSVD_E_INVAL;
    if (prm.precision != HSVD_FP64 && prm.precision != HSVD_MIXED) return HSVD_E_INVAL;
    if (prm.algo != HSVD_AUTO && prm.algo != HSVD_PAIRWISE && prm.algo != HSVD_BLOCK) return HSVD_E_INVAL;
    if (prm.block != 0 && prm.block != block_width() && prm.block != kWideB) return HSVD_E_INVAL;
    if (V && !prm.want_v) return HSVD_E_INVAL;
    const bool mixed = prm.precision == HSVD_MIXED;
    // column blocks of 64: the wide block path, FP64 only
    const bool wide = prm.block == kWideB;
    if (wide && (mixed || prm.algo == HSVD_PAIRWISE)) return HSVD_E_INVAL;
    if (mixed && prm.algo == HSVD_PAIRWISE) return HSVD_E_INVAL;
    if (prm.inner_sweeps < 0 || prm.inner_sweeps > 100) return HSVD_E_INVAL;
    if (prm.persistent < 0 || prm.persistent > 2) return HSVD_E_INVAL;
    const bool full_block = prm.inner_sweeps > 0;
    if (full_block && prm.algo == HSVD_PAIRWISE) return HSVD_E_INVAL;
    // The block path needs at least two blocks of b columns; AUTO takes the
    // autotuner's choice for n's size bucket, else the block path from n >= 512;
    // the mixed path and the full-block method always run blocked.
    const hsvd_ctx::Tune &tn = ctx->tune[size_bucket(n)];
    const bool tuned = prm.algo == HSVD_AUTO && prm.block == 0 && !full_block && tn.valid;
    const bool block = wide || mixed || full_block || prm.algo == HSVD_BLOCK ||
                       (prm.algo == HSVD_AUTO && (tuned ? tn.algo == HSVD_BLOCK : n >= 512));
    const int b = block ? (wide ? kWideB : block_width()) : 0;
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
        // split the Gram's rows so that about 512 workgroups (two per CU; or
        // the tuned number) run per step: longer row runs per column read
        // faster than more, shorter ones (n = 4096: 8 splits of 512 rows
        // 1.15x faster than 16 of 256), and the inner solve sums fewer
        // partial Grams
        const int chunks = ldg / 64;
        const int target = (tuned && tn.wg > 0) ? tn.wg : 512;
        int want = (target + pairs - 1) / pairs;
        want = want < 1 ? 1 : (want > chunks ? chunks : want);
        if (want > 32) want = 32;  // the inner kernels sum at most 32 partial Grams
        rows_per_split = (chunks + want - 1) / want * 64;
        splits = (ldg + rows_per_split - 1) / rows_per_split;
        if (wide) {
            // equal row splits (a power of two dividing ldg / 16) for about 512
            // (pair, split) products per step
            splits = 1;
            while (splits < 16 && pairs * splits < 512 && ldg % (32 * splits) == 0) splits *= 2;
            rows_per_split = ldg / splits;
        }
    }
    const int steps_per_sweep = block ? (prm.ordering == HSVD_ORD_MODMOD ? nb : nb - 1)
                                      : (prm.ordering == HSVD_ORD_MODMOD ? r : r - 1);

    HSVD_TRY(hipSetDevice(ctx->device));
    // the mixed path needs V (to re-orthogonalise and form G X) even when it is not returned
    const bool acc_v = want_v || mixed;
    const Layout L = make_layout(n, r, ldg, acc_v, pairs, splits, block ? 2 * b : 0, mixed);
    hsvd_status s = HSVD_OK;
    void *base = mode.ws;
    if (base) {
        if (L.bytes > mode.ws_cap) return mode.too_big;
    } else {
        s = ensure_ws(ctx, L.bytes);
        if (s != HSVD_OK) return s;
        base = ctx->ws;
    }
    const bool timing = mode.timing;
    if (timing) {
        const int nev = block ? 4 + 4 * steps_per_sweep + 2 : 4;
        s = ensure_events(ctx, (size_t)nev);
        if (s != HSVD_OK) return s;
    }
    const Workspace w = carve(base, L);
    Workspace fin = w;  // what finalize reads (the wide path returns its own buffers)
    hipStream_t st = ctx->stream;
    hipEvent_t *ev = timing ? ctx->events.data() : nullptr;

    // set-up (Alg. 4.2): bordered working copy, V = I, d, rho, steppers, the
    // first sort; the control block tells whether the input is usable
    auto start = [&]() -> hsvd_status {
        HSVD_TRY(launch_zero_ctl(st, w.ctl));
        HSVD_TRY(launch_setup(st, G, lda, n, w, r, ldg, want_v));
        HSVD_TRY(launch_precompute(st, w, r, ldg));
        if (block) HSVD_TRY(launch_block_stepper_init(st, w.S2, nb));
        if (prm.sort) HSVD_TRY(launch_sort(st, w.d, w.rho, w.dtmp, w.rtmp, r, p));
        HSVD_TRY(hipMemcpyAsync(ctx->host_ctl, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
        HSVD_TRY(hipStreamSynchronize(st));
        return HSVD_OK;
    };
    if (timing) HSVD_TRY(hipEventRecord(ev[0], st));
    s = start();
    if (s != HSVD_OK) return s;

    hsvd_status status = HSVD_OK;
    int sweeps = 0, sweeps32 = 0, code = 0, ns_iters = 0, restarted = 0;
    unsigned long long tcol32 = 0;  // touched columns of the FP32 phase (cumulative counter at its end)
    unsigned long long tcol64_base = 0;  // cumulative counter where the FP64 sweeps start
    double maxt_last = 0.0, ns_resid = 0.0;
    long long steps = 0;
    double kms[HSVD_NKERNELS] = {0};
    long long klaunch[HSVD_NKERNELS] = {0};
    long long ktimed[HSVD_NKERNELS] = {0};
    if (ctx->host_ctl->inval) status = HSVD_E_INVAL;
    else if (ctx->host_ctl->rank) status = HSVD_E_RANK;

    bool converged = false;
    long long gstep = 0;
    if (status == HSVD_OK && !block) {
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
        a.maxt = w.maxt;
        a.ctl = w.ctl;
        a.ordering = prm.ordering;
        a.tol = tol;
        a.tthresh = tthresh;
        // The r (or r - 1) dependent step launches of a sweep are captured
        // once as a HIP graph and replayed every sweep (the stepper state
        // lives in device memory and every launch's arguments repeat from
        // sweep to sweep); a step moves only a few MB at moderate n, so the
        // per-launch gap of stream launches is a large share of it.  The
        // sweep runs on the context's capture stream, joined to the caller's
        // stream before and after.
        if (prm.persistent) {
            // every sweep in one persistent launch; the device sorts, reduces
            // and applies the stop rule after each sweep
            PairPersistArgs pa;
            pa.a = a;
            pa.a.step = 0;
            pa.steps = steps_per_sweep;
            pa.max_sweeps = max_sweeps;
            pa.sort = prm.sort ? 1 : 0;
            pa.dataflow = prm.persistent == 1 ? 1 : 0;
            pa.dtmp = w.dtmp;
            pa.rtmp = w.rtmp;
            pa.nact = w.nact;
            pa.ntc = w.ntc;
            pa.ver = w.ver;
            pa.pc = w.pctl;
            int clock_khz = 0;
            HSVD_TRY(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, ctx->device));
            // one wait of a healthy launch lasts at most a step or a sweep's
            // end; 2 s of wall clock means the launch cannot go on
            pa.spin_limit = 2000LL * (clock_khz > 0 ? clock_khz : 100000);
            int grid = 0;
            if (timing) HSVD_TRY(hipEventRecord(ev[2], st));
            const hipError_t le = launch_pair_persist(st, pa, &grid);
            if (le == hipErrorNotSupported || le == hipErrorCooperativeLaunchTooLarge) return HSVD_E_INVAL;
            if (le != hipSuccess) return HSVD_E_DEVICE;
            if (timing) HSVD_TRY(hipEventRecord(ev[3], st));
            HSVD_TRY(hipMemcpyAsync(ctx->host_ctl, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
            HSVD_TRY(hipMemcpyAsync(ctx->host_pctl, w.pctl, sizeof(PersistCtl), hipMemcpyDeviceToHost, st));
            HSVD_TRY(hipStreamSynchronize(st));
            if (ctx->host_pctl->err) return HSVD_E_DEVICE;
            sweeps = ctx->host_pctl->sweeps;
            steps = (long long)sweeps * steps_per_sweep;
            klaunch[HSVD_K_PAIR_STEP] += 1;
            ktimed[HSVD_K_PAIR_STEP] += 1;
            if (timing) {
                float ms = 0.f;
                HSVD_TRY(hipEventElapsedTime(&ms, ev[2], ev[3]));
                kms[HSVD_K_PAIR_STEP] += ms;
            }
            code = ctx->host_ctl->code;
            maxt_last = ctx->host_ctl->maxt;
            if (ctx->host_pctl->stop == 2) status = HSVD_E_RANK;
            else if (ctx->host_pctl->stop == 1) converged = true;
            if (status == HSVD_OK && !converged) status = HSVD_E_NOCONV;
        }
        SweepGraph sg(ctx, st);
        hipStream_t q = st;
        const bool graph = prm.graph && mode.graphs && !prm.persistent;
        if (graph) {
            HSVD_TRY(sg.begin(q));
            for (int k = 0; k < steps_per_sweep; ++k) {
                a.step = k;
                const hipError_t le = launch_pair_step(q, a);
                if (le != hipSuccess) {
                    sg.abort(q);
                    return HSVD_E_DEVICE;
                }
            }
            HSVD_TRY(sg.end(q));
        }
        for (int sw = 0; sw < (prm.persistent ? 0 : max_sweeps); ++sw) {
            if (timing) HSVD_TRY(hipEventRecord(ev[2], q));
            if (graph) {
                HSVD_TRY(hipGraphLaunch(sg.exec, q));
            } else {
                for (int k = 0; k < steps_per_sweep; ++k) {
                    a.step = k;
                    HSVD_TRY(launch_pair_step(q, a));
                }
            }
            if (timing) HSVD_TRY(hipEventRecord(ev[3], q));
            klaunch[HSVD_K_PAIR_STEP] += steps_per_sweep;
            ktimed[HSVD_K_PAIR_STEP] += steps_per_sweep;
            steps += steps_per_sweep;
            if (prm.sort) HSVD_TRY(launch_sort(q, w.d, w.rho, w.dtmp, w.rtmp, r, p));
            HSVD_TRY(launch_sweep_reduce(q, w, r / 2));
            HSVD_TRY(hipMemcpyAsync(ctx->host_ctl, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, q));
            HSVD_TRY(hipStreamSynchronize(q));
            if (timing) {
                float ms = 0.f;
                HSVD_TRY(hipEventElapsedTime(&ms, ev[2], ev[3]));
                kms[HSVD_K_PAIR_STEP] += ms;
            }
            ++sweeps;
            code = ctx->host_ctl->code;
            maxt_last = ctx->host_ctl->maxt;
            if (ctx->host_ctl->rank) {
                status = HSVD_E_RANK;
                break;
            }
            if ((code & 2) == 0) {  // eq. (4.2): codes 00 and 01 stop the process
                converged = true;
                break;
            }
        }
        if (!prm.persistent && status == HSVD_OK && !converged) status = HSVD_E_NOCONV;
    } else if (status == HSVD_OK) {
        SweepResult last = {0, 0.0, false};
        bool finished = false;
        if (mixed) {
            // FP32 sweeps on FP32 copies of G and V.
            HSVD_TRY(launch_to_fp32(st, w.G, w.G32, w.V32, ldg, r));
            BlockArgsT<float> fa;
            fa.G = w.G32;
            fa.V = w.V32;
            fa.ldg = ldg;
            fa.r = r;
            fa.p = p;
            fa.nb = nb;
            fa.rho = w.rho;
            fa.ordering = prm.ordering;
            fa.partial = w.P32;
            fa.splits = splits;
            fa.rows_per_split = rows_per_split;
            fa.W = w.W32;
            fa.active = w.active;
            fa.C = w.C;
            fa.nrot = w.nrot;
            fa.nskip = w.nskip;
            fa.nact = w.nact;
            fa.ntc = w.ntc;
            fa.maxt = w.maxt;
            fa.ctl = w.ctl;
            // the FP32 Gram resolves cosines down to about sqrt(r) FP32 epsilons
            const double tol32 = fmax(tol, sqrt((double)r) * 0x1p-23);
            fa.tol = tol32;
            fa.tthresh = sqrt(tol32) / 2.0;
            fa.inner_sweeps = prm.inner_sweeps;
            double prev = 1.0, prev_frac = 1.0;
            unsigned long long rot0 = 0, skip0 = 0;  // the counters start at zero with the solve
            int sw32 = 0;
            // Leave FP32 when the largest tangent of a sweep is at the FP32
            // resolution (<= 3e-4 ~ sqrt(eps32)), when it stagnates (falls by
            // less than 4x once below 0.1), when FP32 itself converged, or by
            // the fraction f of the sweep's pair visits that rotated: f < 1/100
            // (the tail of a geometric decline; the first FP64 sweep rotates
            // nearly every pair again in any case), or f <= 1/3 while falling by
            // less than a quarter per sweep (a slow decline: the remaining
            // rotations are below what FP32 resolves and the FP64 sweeps redo
            // them).
            auto done32 = [&](const SweepResult &sr) {
                const unsigned long long rot = ctx->host_ctl->rot, skip = ctx->host_ctl->skip;
                const double dr = (double)(rot - rot0), ds = (double)(skip - skip0);
                const double frac = dr + ds > 0.0 ? dr / (dr + ds) : 0.0;
                rot0 = rot;
                skip0 = skip;
                const bool stop = sr.maxt <= 3e-4 || (sr.code & 2) == 0 ||
                                  (sr.maxt < 0.1 && sr.maxt > 0.25 * prev) || frac < 0.01 ||
                                  (frac <= 1.0 / 3.0 && frac >= 0.75 * prev_frac);
                prev = sr.maxt;
                prev_frac = frac;
                return stop;
            };
            status = block_sweeps<float>(ctx, w, fa, w.G32, pairs, steps_per_sweep, max_sweeps, prm.sort != 0, r,
                                         p, ldg, gstep, HSVD_K_BLOCK_GRAM32, kms, klaunch, ktimed, sw32, steps, last,
                                         finished, timing, done32);
            sweeps32 = sw32;
            tcol32 = ctx->host_ctl->tcol;
            tcol64_base = tcol32;
            if (status == HSVD_E_DEVICE) return status;
            // A rank flag in an FP32 sweep may come from the FP32 Gram alone
            // (it resolves S - |w| of a hyperbolic pair only to about sqrt(r)
            // FP32 epsilons), and V32 is then no iterate to refine: the solve
            // starts again from G in FP64, where a rank failure is final.
            bool restart = status == HSVD_E_RANK;
            if (status == HSVD_OK) {
                // back to FP64: X = J-orthogonalised V32, G1 = G X, V0 = X
                if (timing) HSVD_TRY(hipEventRecord(ev[2], st));
                HSVD_TRY(launch_promote(st, w.V32, w.V, ldg, r));
                s = reorthogonalise(ctx, w, n, r, p, ldg, ns_iters, ns_resid);
                if (s != HSVD_OK) return s;
                if (timing) {
                    HSVD_TRY(hipEventRecord(ev[3], st));
                    HSVD_TRY(hipStreamSynchronize(st));
                    float ms = 0.f;
                    HSVD_TRY(hipEventElapsedTime(&ms, ev[2], ev[3]));
                    kms[HSVD_K_REORTH] += ms;
                    ktimed[HSVD_K_REORTH] += 1;
                }
                klaunch[HSVD_K_REORTH] += 1;
                // X not J-orthogonal to working accuracy (the iteration left its
                // basin, stalled, or hit its cap): G X and V0 = X would carry
                // that error into the result, so start again in FP64 as well
                restart = !(ns_resid <= reorth_accept_bound(prm, n));
                if (!restart) {
                    HSVD_TRY(launch_colnorm_pos<double>(st, w.G, ldg, w.rho, w.d, r));
                    if (prm.sort) HSVD_TRY(launch_sort(st, w.d, w.rho, w.dtmp, w.rtmp, r, p));
                }
            }
            if (restart) {
                // the same launches as a plain FP64 solve from here on (the
                // stepper restarts with the step count), so the result is that
                // solve's
                restarted = 1;
                gstep = 0;
                tcol64_base = 0;
                status = HSVD_OK;
                s = start();
                if (s != HSVD_OK) return s;
                if (ctx->host_ctl->inval) status = HSVD_E_INVAL;
                else if (ctx->host_ctl->rank) status = HSVD_E_RANK;
            }
        }
        if (status == HSVD_OK && wide) {
            double *fG = nullptr, *fV = nullptr;
            int *frho = nullptr;
            status = wide_sweeps(ctx, w, r, p, ldg, nb, splits, prm.ordering, want_v, prm.sort != 0, tol, tthresh,
                                 prm.inner_sweeps, max_sweeps, timing, kms, klaunch, ktimed, sweeps, steps, last,
                                 finished, fG, fV, frho);
            code = last.code;
            maxt_last = last.maxt;
            if (status == HSVD_OK && !finished) status = HSVD_E_NOCONV;
            fin.G = fG;
            fin.V = fV;
            fin.rho = frho;
        } else if (status == HSVD_OK) {
            BlockArgs ba;
            ba.G = w.G;
            ba.V = want_v ? w.V : nullptr;  // the mixed path keeps V only when it is returned
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
            ba.ntc = w.ntc;
            ba.maxt = w.maxt;
            ba.ctl = w.ctl;
            ba.tol = tol;
            ba.tthresh = tthresh;
            ba.inner_sweeps = prm.inner_sweeps;
            auto done64 = [](const SweepResult &sr) { return (sr.code & 2) == 0; };  // eq. (4.2)
            status = block_sweeps<double>(ctx, w, ba, w.G, pairs, steps_per_sweep, max_sweeps, prm.sort != 0, r, p,
                                          ldg, gstep, HSVD_K_BLOCK_GRAM, kms, klaunch, ktimed, sweeps, steps, last,
                                          finished, timing, done64);
            code = last.code;
            maxt_last = last.maxt;
            if (status == HSVD_OK && !finished) status = HSVD_E_NOCONV;
        }
        if (status == HSVD_E_DEVICE) return status;
    }

    HSVD_TRY(launch_finalize(st, fin, n, r, p, ldg, sigma, U, ldu, V, ldv, lambda, perm));
    if (timing) HSVD_TRY(hipEventRecord(ev[1], st));
    HSVD_TRY(hipStreamSynchronize(st));
    if (info) {
        float ms = 0.f;
        if (timing) hipEventElapsedTime(&ms, ev[0], ev[1]);
        info->status = status;
        info->sweeps = sweeps;
        info->sweeps_fp32 = sweeps32;
        info->reorth_iters = ns_iters;
        info->reorth_resid = ns_resid;
        info->fp64_restart = restarted;
        info->max_t_last = maxt_last;
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
            info->kernel_timed[q] = ktimed[q];
        }
        if (!block) {
            // a rotated pair reads and writes two columns of G (and of V); a
            // skipped pair reads two columns of G; flops: dot 2, update 6 and
            // new norms 4 per row for G, update 6 per row for V
            const double rot = (double)info->rotations, skp = (double)info->skips;
            info->kernel_bytes[HSVD_K_PAIR_STEP] = rot * 32.0 * rows * vmul + skp * 16.0 * rows;
            info->kernel_flops[HSVD_K_PAIR_STEP] = rot * (12.0 + 6.0 * (vmul - 1.0)) * rows + skp * 2.0 * rows;
        } else {
            // per block pair and step: the Gram reads 2b columns and issues the
            // upper 10 of the 16 tiles of the (2b)^2 x rows product; the update
            // must read and write only the columns of G (and of V) that a
            // rotation touched, each the product of 2b columns with a column of
            // W (2b x rows multiply-adds).  The inner launch's own traffic
            // (partial Grams in, W out) belongs to splitting the Gram's rows,
            // not to the method, and is not counted.  The FP32 phase of the
            // mixed path always carries V.
            const double b2 = 2.0 * b;
            const double tc_all = (double)ctx->host_ctl->tcol;
            const double st64 = (double)klaunch[HSVD_K_BLOCK_GRAM], st32 = (double)klaunch[HSVD_K_BLOCK_GRAM32];
            for (int prec = 0; prec < 2; ++prec) {
                const int kb = prec == 0 ? HSVD_K_BLOCK_GRAM : HSVD_K_BLOCK_GRAM32;
                const double esz = prec == 0 ? 8.0 : 4.0;
                const double visits = (prec == 0 ? st64 : st32) * pairs;
                const double tcols = prec == 0 ? tc_all - (double)tcol64_base : (double)tcol32;
                const double vm = prec == 0 ? vmul : 2.0;
                // with V carried by the block-oriented method, V's half of the
                // update runs inside the inner launches and is counted there
                // (the wide path updates V in its update launch, and its Gram
                // forms the whole (2b)^2 product)
                const double vin = (vm > 1.0 && prm.inner_sweeps == 0 && !wide) ? 1.0 : 0.0;
                info->kernel_bytes[kb] = visits * esz * b2 * rows;
                info->kernel_flops[kb] = visits * 2.0 * (wide ? 1.0 : 10.0 / 16.0) * b2 * b2 * rows;
                info->kernel_bytes[kb + 1] = vin * tcols * 2.0 * esz * rows;
                info->kernel_flops[kb + 1] = vin * tcols * 2.0 * b2 * rows;
                info->kernel_bytes[kb + 2] = tcols * 2.0 * esz * rows * (vm - vin);
                info->kernel_flops[kb + 2] = tcols * 2.0 * b2 * rows * (vm - vin);
            }
            if (mixed && klaunch[HSVD_K_REORTH] > 0) {
                // X^T J X formed iters + 1 times (upper tiles only: a fraction
                // (T + 1) / 2T of the product with T tiles per side), X T iters
                // times, G X once; each product reads two r x r matrices and
                // writes one
                const double rr = (double)r, nt = (double)((r + 127) / 128);
                const double full = 2.0 * rr * rr * rr;
                info->kernel_flops[HSVD_K_REORTH] =
                    (ns_iters + 1.0) * full * (nt + 1.0) / (2.0 * nt) + (ns_iters + 1.0) * full;
                info->kernel_bytes[HSVD_K_REORTH] = (2.0 * ns_iters + 2.0) * 3.0 * 8.0 * rr * rr;
            }
        }
    }
    return status;
}

size_t take_bytes(size_t &o, size_t bytes)
{
    const size_t at = o;
    o = (o + bytes + 255) / 256 * 256;
    return at;
}

// Device buffer of the context for the partitioned solve (outside the solver's workspace).
hsvd_status ensure_aux(hsvd_ctx *ctx, size_t bytes)
{
    if (ctx->aux_bytes >= bytes) return HSVD_OK;
    if (ctx->aux) {
        HSVD_TRY(hipStreamSynchronize(ctx->stream));
        hipFree(ctx->aux);
        ctx->aux = nullptr;
        ctx->aux_bytes = 0;
    }
    if (hipMalloc(&ctx->aux, bytes) != hipSuccess) return HSVD_E_NOMEM;
    ctx->aux_bytes = bytes;
    return HSVD_OK;
}

}  // namespace

extern "C" hsvd_status hsvd_solve(hsvd_ctx *ctx, const double *G, int lda, const signed char *jsig, int n, int p,
                                  const hsvd_params *prm_in, double *sigma, double *U, int ldu, double *V, int ldv,
                                  double *lambda, int *perm, hsvd_info *info)
{
    if (info) memset(info, 0, sizeof(*info));
    if (!ctx || !G || !sigma || n < 1 || p < 0 || p > n || lda < n) return HSVD_E_INVAL;
    if (U && ldu < n) return HSVD_E_INVAL;
    if (V && ldv < n) return HSVD_E_INVAL;
    hsvd_params prm;
    if (prm_in) prm = *prm_in;
    else hsvd_default_params(&prm);
    const SolveMode mode;
    if (!jsig) return solve_canonical(ctx, G, lda, n, p, prm, sigma, U, ldu, V, ldv, lambda, perm, info, mode);
    HSVD_TRY(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    std::vector<signed char> hj(n);
    HSVD_TRY(hipMemcpyAsync(hj.data(), jsig, n, hipMemcpyDeviceToHost, st));
    HSVD_TRY(hipStreamSynchronize(st));
    // stable partition: the +1 columns first, each class in input order
    std::vector<int> pi;
    pi.reserve(n);
    for (int c = 0; c < n; ++c) {
        if (hj[c] != 1 && hj[c] != -1) return HSVD_E_INVAL;
        if (hj[c] == 1) pi.push_back(c);
    }
    if ((int)pi.size() != p) return HSVD_E_INVAL;
    bool canonical = true;
    for (int c = 0; c < p; ++c) canonical = canonical && pi[c] == c;
    if (canonical) return solve_canonical(ctx, G, lda, n, p, prm, sigma, U, ldu, V, ldv, lambda, perm, info, mode);
    for (int c = 0; c < n; ++c)
        if (hj[c] == -1) pi.push_back(c);
    // aux: pi, Gp, sigma_p, lambda_p, perm_p, U_p, V_p
    size_t o = 0;
    const size_t nn = (size_t)n * n;
    const size_t o_pi = take_bytes(o, sizeof(int) * n), o_Gp = take_bytes(o, sizeof(double) * nn);
    const size_t o_s = take_bytes(o, sizeof(double) * n), o_l = take_bytes(o, sizeof(double) * n);
    const size_t o_pm = take_bytes(o, sizeof(int) * n), o_U = take_bytes(o, U ? sizeof(double) * nn : 0);
    const size_t o_V = take_bytes(o, V ? sizeof(double) * nn : 0);
    hsvd_status s = ensure_aux(ctx, o);
    if (s != HSVD_OK) return s;
    char *a = static_cast<char *>(ctx->aux);
    int *dpi = reinterpret_cast<int *>(a + o_pi);
    double *Gp = reinterpret_cast<double *>(a + o_Gp);
    double *sp = reinterpret_cast<double *>(a + o_s), *lp = reinterpret_cast<double *>(a + o_l);
    int *pmp = reinterpret_cast<int *>(a + o_pm);
    double *Up = U ? reinterpret_cast<double *>(a + o_U) : nullptr;
    double *Vp = V ? reinterpret_cast<double *>(a + o_V) : nullptr;
    HSVD_TRY(hipMemcpyAsync(dpi, pi.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
    HSVD_TRY(launch_gather_cols(st, G, lda, dpi, Gp, n));
    s = solve_canonical(ctx, Gp, n, n, p, prm, sp, Up, n, Vp, n, lp, pmp, info, mode);
    if (s == HSVD_E_INVAL || s == HSVD_E_DEVICE || s == HSVD_E_NOMEM) return s;
    HSVD_TRY(launch_scatter_outputs(st, dpi, n, sp, Up, Vp, lp, pmp, sigma, U, ldu, V, ldv, lambda, perm));
    HSVD_TRY(hipStreamSynchronize(st));
    return s;
}

extern "C" hsvd_status hsvd_solve_noalloc(hsvd_ctx *ctx, const double *G, int lda, int n, int p,
                                          const hsvd_params *prm_in, double *sigma, double *U, int ldu, double *V,
                                          int ldv, double *lambda, int *perm, hsvd_info *info)
{
    if (info) memset(info, 0, sizeof(*info));
    if (!ctx || !G || !sigma || n < 1 || p < 0 || p > n || lda < n) return HSVD_E_INVAL;
    hsvd_params prm;
    if (prm_in) prm = *prm_in;
    else hsvd_default_params(&prm);
    // the persistent pairwise kernel is a cooperative launch, which the
    // runtime may back with allocations of its own
    if (prm.persistent != 0) return HSVD_E_INVAL;
    HSVD_TRY(hipSetDevice(ctx->device));
    void *ptr = scratch_address(ctx->device);
    if (!ptr) return HSVD_E_DEVICE;
    SolveMode mode;
    mode.ws = ptr;
    mode.ws_cap = HSVD_NOALLOC_BYTES;
    mode.timing = false;  // no events (created on demand otherwise)
    mode.graphs = false;  // no graph capture (instantiation allocates)
    mode.too_big = HSVD_E_SIZE;
    return solve_canonical(ctx, G, lda, n, p, prm, sigma, U, ldu, V, ldv, lambda, perm, info, mode);
}

extern "C" hsvd_status hsvd_autotune(hsvd_ctx *ctx, int n, int *best_algo, int *best_wg)
{
    if (!ctx || n < 2 || n > kMaxOrder - 2) return HSVD_E_INVAL;
    HSVD_TRY(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    // synthetic problem and outputs in the auxiliary buffer
    size_t o = 0;
    const size_t nn = (size_t)n * n;
    const size_t o_G = take_bytes(o, sizeof(double) * nn), o_s = take_bytes(o, sizeof(double) * n);
    const hsvd_status sa = ensure_aux(ctx, o);
    if (sa != HSVD_OK) return sa;
    double *G = reinterpret_cast<double *>(static_cast<char *>(ctx->aux) + o_G);
    double *sig = reinterpret_cast<double *>(static_cast<char *>(ctx->aux) + o_s);
    HSVD_TRY(launch_synth(st, G, n, 0x5EEDull + (unsigned long long)n));
    struct Cand {
        int algo, wg;
    } cands[5] = {{HSVD_PAIRWISE, 0}, {HSVD_BLOCK, 256}, {HSVD_BLOCK, 512}, {HSVD_BLOCK, 1024}, {HSVD_BLOCK, 2048}};
    const int bucket = size_bucket(n);
    const hsvd_ctx::Tune saved = ctx->tune[bucket];
    double best = 1e300;
    int ba = HSVD_BLOCK, bw = 1024;
    for (const Cand &c : cands) {
        hsvd_params prm;
        hsvd_default_params(&prm);
        prm.want_v = 1;
        prm.max_sweeps = 2;
        ctx->tune[bucket].valid = 1;
        ctx->tune[bucket].algo = c.algo;
        ctx->tune[bucket].wg = c.wg;
        hsvd_info info;
        double t = 0.0;
        for (int rep = 0; rep < 2; ++rep) {  // the first run also warms up
            const hsvd_status s = hsvd_solve(ctx, G, n, nullptr, n, n / 2, &prm, sig, nullptr, n, nullptr, n,
                                             nullptr, nullptr, &info);
            if (s != HSVD_OK && s != HSVD_E_NOCONV) {
                ctx->tune[bucket] = saved;
                return s;
            }
            t = info.ms_total;
        }
        if (t < best) {
            best = t;
            ba = c.algo;
            bw = c.wg;
        }
    }
    ctx->tune[bucket].valid = 1;
    ctx->tune[bucket].algo = ba;
    ctx->tune[bucket].wg = bw;
    tune_save(ctx);
    if (best_algo) *best_algo = ba;
    if (best_wg) *best_wg = bw;
    return HSVD_OK;
}

// Autotuner of the persistent batched kernel: the workgroup width (256, 512
// or 1024 threads per problem) for the bucket of the largest order among the
// given problems, timed on a sample of them with seeded synthetic entries.
extern "C" hsvd_status hsvd_autotune_batched(hsvd_ctx *ctx, int batch, const int *n_in, const int *p_in,
                                             int *best_threads, float *ms_out)
{
    if (!ctx || batch < 1 || !n_in || !p_in) return HSVD_E_INVAL;
    HSVD_TRY(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    std::vector<int> n(batch), p(batch);
    HSVD_TRY(hipMemcpyAsync(n.data(), n_in, sizeof(int) * batch, hipMemcpyDefault, st));
    HSVD_TRY(hipMemcpyAsync(p.data(), p_in, sizeof(int) * batch, hipMemcpyDefault, st));
    HSVD_TRY(hipStreamSynchronize(st));
    // a sample of at most 4096 problems, every k-th, and only those the
    // persistent kernel takes
    const int stride = (batch + 4095) / 4096;
    std::vector<int> sn, sp;
    for (int k = 0; k < batch; k += stride) {
        if (n[k] < 1 || n[k] > 1024 || p[k] < 0 || p[k] > n[k]) return HSVD_E_INVAL;
        if (n[k] <= kPersistMaxOrder) {
            sn.push_back(n[k]);
            sp.push_back(p[k]);
        }
    }
    if (sn.empty()) return HSVD_E_INVAL;
    const int K = (int)sn.size();
    int nmax = 0;
    std::vector<long long> off(K), voff(K);
    long long tot = 0, totv = 0;
    for (int k = 0; k < K; ++k) {
        off[k] = tot;
        voff[k] = totv;
        tot += (long long)sn[k] * sn[k];
        totv += sn[k];
        nmax = std::max(nmax, sn[k]);
    }
    size_t o = 0;
    const size_t o_G = take_bytes(o, sizeof(double) * tot), o_U = take_bytes(o, sizeof(double) * tot);
    const size_t o_V = take_bytes(o, sizeof(double) * tot), o_s = take_bytes(o, sizeof(double) * totv);
    const hsvd_status sa = ensure_aux(ctx, o);
    if (sa != HSVD_OK) return sa;
    char *base = static_cast<char *>(ctx->aux);
    double *G = reinterpret_cast<double *>(base + o_G);
    for (int k = 0; k < K; ++k) HSVD_TRY(launch_synth(st, G + off[k], sn[k], 0xBA7C4ull + (unsigned long long)k));
    // two events of its own, past the ones hsvd_solve_batched uses (handles,
    // not pointers into the context's list, which that call may grow)
    const size_t nev = 4 + 4 * 1024 / block_width();
    hsvd_status se = ensure_events(ctx, nev + 2);
    if (se != HSVD_OK) return se;
    const hipEvent_t ev[2] = {ctx->events[nev], ctx->events[nev + 1]};
    hsvd_params prm;
    hsvd_default_params(&prm);
    prm.batch_mode = 0;  // the widths are the persistent launch's
    const int bucket = std::min(3, (nmax - 1) / 64);
    const int saved = ctx->persist_threads[bucket];
    const int cands[3] = {256, 512, 1024};
    int best = kPersistDefaultThreads;
    float best_ms = 1e30f;
    for (int ci = 0; ci < 3; ++ci) {
        ctx->persist_threads[bucket] = cands[ci];
        float ms = 0.f;
        for (int rep = 0; rep < 2; ++rep) {  // the first run also warms up
            HSVD_TRY(hipEventRecord(ev[0], st));
            const hsvd_status s =
                hsvd_solve_batched(ctx, K, sn.data(), sp.data(), off.data(), voff.data(), G, &prm,
                                   reinterpret_cast<double *>(base + o_s), reinterpret_cast<double *>(base + o_U),
                                   reinterpret_cast<double *>(base + o_V), nullptr, nullptr);
            if (s != HSVD_OK && s != HSVD_E_NOCONV) {
                ctx->persist_threads[bucket] = saved;
                return s;
            }
            HSVD_TRY(hipEventRecord(ev[1], st));
            HSVD_TRY(hipEventSynchronize(ev[1]));
            HSVD_TRY(hipEventElapsedTime(&ms, ev[0], ev[1]));
        }
        if (ms_out) ms_out[ci] = ms;
        if (ms < best_ms) {
            best_ms = ms;
            best = cands[ci];
        }
    }
    ctx->persist_threads[bucket] = best;
    // The sweep schedule per precision, with the chosen width: one persistent
    // launch against launches grouped by order, timed on the problems whose
    // schedule it decides (n <= kPersistMaxOrder), all of them up to 16384
    // (every k-th beyond): the grouped launches gain with the number of
    // problems per group, so a small sample would not tell.
    std::vector<int> an, ap;
    {
        int small = 0;
        for (int k = 0; k < batch; ++k) small += n[k] <= kPersistMaxOrder ? 1 : 0;
        const int stride2 = (small + 16383) / 16384;
        int seen = 0;
        for (int k = 0; k < batch; ++k) {
            if (n[k] > kPersistMaxOrder) continue;
            if (seen++ % stride2 == 0) {
                an.push_back(n[k]);
                ap.push_back(p[k]);
            }
        }
    }
    const int A = (int)an.size();
    std::vector<long long> aoff(A), avoff(A);
    long long atot = 0, atotv = 0;
    for (int k = 0; k < A; ++k) {
        aoff[k] = atot;
        avoff[k] = atotv;
        atot += (long long)an[k] * an[k];
        atotv += an[k];
    }
    size_t oa = 0;
    const size_t a_G = take_bytes(oa, sizeof(double) * atot), a_U = take_bytes(oa, sizeof(double) * atot);
    const size_t a_V = take_bytes(oa, sizeof(double) * atot), a_s = take_bytes(oa, sizeof(double) * atotv);
    const hsvd_status sa2 = ensure_aux(ctx, oa);
    if (sa2 != HSVD_OK) return sa2;
    char *abase = static_cast<char *>(ctx->aux);
    double *AG = reinterpret_cast<double *>(abase + a_G);
    for (int k = 0; k < A; ++k)
        HSVD_TRY(launch_synth(st, AG + aoff[k], an[k], 0x5C4EDull + (unsigned long long)k));
    for (int pr = 0; pr < 2; ++pr) {
        float sched_ms[2] = {0.f, 0.f};
        for (int mode = 0; mode < 2; ++mode) {
            hsvd_params q = prm;
            q.precision = pr ? HSVD_MIXED : HSVD_FP64;
            q.batch_mode = mode;
            for (int rep = 0; rep < 2; ++rep) {  // the first run also warms up
                HSVD_TRY(hipEventRecord(ev[0], st));
                const hsvd_status s = hsvd_solve_batched(
                    ctx, A, an.data(), ap.data(), aoff.data(), avoff.data(), AG, &q,
                    reinterpret_cast<double *>(abase + a_s), reinterpret_cast<double *>(abase + a_U),
                    reinterpret_cast<double *>(abase + a_V), nullptr, nullptr);
                if (s != HSVD_OK && s != HSVD_E_NOCONV) return s;
                HSVD_TRY(hipEventRecord(ev[1], st));
                HSVD_TRY(hipEventSynchronize(ev[1]));
                HSVD_TRY(hipEventElapsedTime(&sched_ms[mode], ev[0], ev[1]));
            }
        }
        ctx->batch_sched[pr] = sched_ms[1] < sched_ms[0] ? 1 : 0;
    }
    tune_save(ctx);
    if (best_threads) *best_threads = best;
    return HSVD_OK;
}

extern "C" hsvd_status hsvd_batched_schedule(const hsvd_ctx *ctx, int precision, int *mode)
{
    if (!ctx || !mode || (precision != HSVD_FP64 && precision != HSVD_MIXED)) return HSVD_E_INVAL;
    *mode = ctx->batch_sched[precision == HSVD_MIXED ? 1 : 0];
    return HSVD_OK;
}

// FP32 phase of a batched mixed solve for one group, then the
// J-re-orthogonalisation of each problem's V and G1 = G X -- the steps of a
// single mixed solve, per problem.  FP32 block sweeps run until every problem
// has left FP32 by its own switch rule (a problem out of FP32 is skipped by
// the later FP32 launches); the Newton-Schulz iteration runs on the whole
// group with the batched FP64 MFMA products, each problem applying its
// corrections until its own residual stops falling quadratically.  The FP64
// sweeps then start from (G1, V0 = X), or from G for a problem that restarts
// (rank flag in its FP32 phase, or a final residual above the accepted one).
static hsvd_status batch_mixed_phase(hsvd_ctx *ctx, hipStream_t st, const BatchGroup &g, const BatchMixed &m,
                                     const BlockArgsT<double> &ba, int4 *S2, int pairs, int steps_per_sweep,
                                     int max_sweeps, bool sort, long long &gstep, int *host_active, int &sweeps32,
                                     const double *Gin)
{
    HSVD_TRY(launch_batch_mixed_init(st, g, m));
    BlockArgsT<float> fa;
    fa.G = m.G32;
    fa.V = m.V32;
    fa.ldg = ba.ldg;
    fa.r = ba.r;
    fa.p = 0;
    fa.nb = ba.nb;
    fa.rho = ba.rho;
    fa.ordering = ba.ordering;
    // the FP32 partial Grams and W in the space of the FP64 ones
    fa.partial = reinterpret_cast<float *>(ba.partial);
    fa.splits = ba.splits;
    fa.rows_per_split = ba.rows_per_split;
    fa.W = reinterpret_cast<float *>(ba.W);
    fa.active = ba.active;
    fa.C = ba.C;
    fa.nrot = ba.nrot;
    fa.nskip = ba.nskip;
    fa.nact = ba.nact;
    fa.ntc = ba.ntc;
    fa.maxt = ba.maxt;
    fa.ctl = ba.ctl;
    fa.tol = 0.0;
    fa.tthresh = 0.0;
    fa.inner_sweeps = ba.inner_sweeps;
    fa.nprob = ba.nprob;
    fa.done = m.done32;
    fa.pvec = ba.pvec;
    fa.tolvec = m.tol32;
    fa.tthvec = m.tth32;
    BatchGroup g32 = g;
    g32.done = m.done32;  // the sort of the FP32 phase skips problems out of it
    sweeps32 = 0;
    for (int sw = 0; sw < max_sweeps; ++sw) {
        for (int k = 0; k < steps_per_sweep; ++k, ++gstep) {
            fa.step = k;
            fa.S_in = S2 + (gstep & 1) * pairs;
            fa.S_out = S2 + ((gstep + 1) & 1) * pairs;
            HSVD_TRY(launch_block_gram<float>(st, fa));
            HSVD_TRY(launch_block_inner<float>(st, fa));
            HSVD_TRY(launch_block_update<float>(st, fa));
        }
        HSVD_TRY(launch_batch_colnorm32(st, g, m));
        if (sort) HSVD_TRY(launch_batch_sort(st, g32));
        HSVD_TRY(launch_batch_decide32(st, g, m));
        HSVD_TRY(hipMemcpyAsync(host_active, g.active_count, sizeof(int), hipMemcpyDeviceToHost, st));
        HSVD_TRY(hipStreamSynchronize(st));
        ++sweeps32;
        if (*host_active == 0) break;
    }
    // V = V32 promoted; Newton-Schulz X <- X (3I - J X^T J X) / 2 per problem,
    // on the FP64 MFMA products with the problem in blockIdx.z
    HSVD_TRY(launch_batch_promote(st, g, m));
    const int r = g.r, ld = g.ldg;
    const long long mat = (long long)g.ldg * g.r;
    GemmArgs sy;  // T2 = X^T J X for the problems still iterating
    sy.A = g.V;
    sy.B = g.V;
    sy.C = m.T2;
    sy.M = sy.N = sy.K = r;
    sy.lda = sy.ldb = sy.ldc = ld;
    sy.sa = sy.sb = sy.sc = mat;
    sy.pvec = g.p;
    sy.flag = m.nsdone;
    sy.want = 0;
    GemmArgs xt = sy;  // T1 = X T2 where the correction applies
    xt.B = m.T2;
    xt.C = m.T1;
    xt.pvec = nullptr;
    xt.flag = m.apply;
    xt.want = 1;
    for (int it = 0; it <= 6; ++it) {
        HSVD_TRY(launch_gemm(st, sy, g.nprob, true, true, true));
        HSVD_TRY(launch_batch_ns_form(st, g, m));  // T2 = (3I - J X^T J X) / 2, residuals
        HSVD_TRY(launch_batch_ns_decide(st, g, m, it, it == 6));
        HSVD_TRY(hipMemcpyAsync(host_active, g.active_count, sizeof(int), hipMemcpyDeviceToHost, st));
        HSVD_TRY(hipStreamSynchronize(st));
        if (*host_active == 0) break;
        HSVD_TRY(launch_gemm(st, xt, g.nprob, false, false, false));
        HSVD_TRY(launch_batch_copy_if(st, g, m.T1, g.V, m.apply, false));
    }
    // problems whose X is not J-orthogonal to working accuracy (or whose FP32
    // phase saw a rank flag) restart from G in FP64; the others go on from
    // G1 = G X (apply marks them)
    HSVD_TRY(launch_batch_ns_accept(st, g, m));
    GemmArgs gx = sy;
    gx.A = g.G;
    gx.B = g.V;
    gx.C = m.T1;
    gx.pvec = nullptr;
    gx.flag = m.apply;
    gx.want = 1;
    HSVD_TRY(launch_gemm(st, gx, g.nprob, false, false, false));
    HSVD_TRY(launch_batch_copy_if(st, g, m.T1, g.G, m.apply, false));
    BatchGroup gr = g;
    gr.only = m.restart;
    HSVD_TRY(launch_batch_setup(st, gr, Gin, true));
    // the kept diagonal of G1 and the sort, as after a sweep
    HSVD_TRY(launch_batch_colnorm(st, g, false));
    if (sort) HSVD_TRY(launch_batch_sort(st, g));
    return HSVD_OK;
}

// The problems `ids` (FP64, block-oriented, n <= kPersistMaxOrder) in one
// persistent launch: a work queue of the problem indices, largest n first
// (the longest solves start first; the short ones fill in at the end), one
// workgroup slot of device memory per resident workgroup, per-problem results
// read back into pinfo.  With prm.graph the queue reset and the launch are
// captured and replayed as one graph.
static hsvd_status batch_persistent(hsvd_ctx *ctx, hipStream_t st, const std::vector<int> &ids, const int *n,
                                    const int *p, const long long *off, const long long *voff, const double *G,
                                    const hsvd_params &prm, int max_sweeps, bool want_v, double *sigma, double *U,
                                    double *V, double *lambda, std::vector<hsvd_info> &pinfo)
{
    const int K = (int)ids.size();
    if (K == 0) return HSVD_OK;
    const int batch = (int)pinfo.size();
    int cus = 0;
    HSVD_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    int nmax = 0;
    for (int k : ids) nmax = std::max(nmax, n[k]);
    const int bucket = std::min(3, (nmax - 1) / 64);
    const int threads = ctx->persist_threads[bucket] ? ctx->persist_threads[bucket] : kPersistDefaultThreads;
    const int per_cu = persist_blocks_per_cu(threads);
    if (per_cu < 1 || cus < 1) return HSVD_E_DEVICE;
    const int wgs = std::min(K, per_cu * cus);
    // the work queue: problem indices by n, largest first (stable)
    std::vector<int> order(ids);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return n[x] > n[y]; });
    size_t o = 0;
    const size_t o_order = take_bytes(o, sizeof(int) * K), o_next = take_bytes(o, sizeof(int));
    const size_t o_n = take_bytes(o, sizeof(int) * batch), o_p = take_bytes(o, sizeof(int) * batch);
    const size_t o_off = take_bytes(o, sizeof(long long) * batch), o_voff = take_bytes(o, sizeof(long long) * batch);
    const size_t o_st = take_bytes(o, sizeof(int) * batch), o_sw = take_bytes(o, sizeof(int) * batch);
    const size_t o_code = take_bytes(o, sizeof(int) * batch), o_mt = take_bytes(o, sizeof(double) * batch);
    const size_t o_rot = take_bytes(o, sizeof(unsigned long long) * batch);
    const size_t o_skip = take_bytes(o, sizeof(unsigned long long) * batch);
    const size_t o_act = take_bytes(o, sizeof(unsigned long long) * batch);
    const size_t o_s32 = take_bytes(o, sizeof(int) * batch), o_ni = take_bytes(o, sizeof(int) * batch);
    const size_t o_rs = take_bytes(o, sizeof(int) * batch), o_nr = take_bytes(o, sizeof(double) * batch);
    const size_t o_slots = take_bytes(o, persist_slot_bytes() * (size_t)wgs);
    hsvd_status s = ensure_ws(ctx, o);
    if (s != HSVD_OK) return s;
    char *base = static_cast<char *>(ctx->ws);
    HSVD_TRY(hipMemcpyAsync(base + o_order, order.data(), sizeof(int) * K, hipMemcpyHostToDevice, st));
    HSVD_TRY(hipMemcpyAsync(base + o_n, n, sizeof(int) * batch, hipMemcpyHostToDevice, st));
    HSVD_TRY(hipMemcpyAsync(base + o_p, p, sizeof(int) * batch, hipMemcpyHostToDevice, st));
    HSVD_TRY(hipMemcpyAsync(base + o_off, off, sizeof(long long) * batch, hipMemcpyHostToDevice, st));
    HSVD_TRY(hipMemcpyAsync(base + o_voff, voff, sizeof(long long) * batch, hipMemcpyHostToDevice, st));
    PersistArgs pa;
    pa.batch = K;
    pa.order = reinterpret_cast<int *>(base + o_order);
    pa.next = reinterpret_cast<int *>(base + o_next);
    pa.n = reinterpret_cast<int *>(base + o_n);
    pa.p = reinterpret_cast<int *>(base + o_p);
    pa.off = reinterpret_cast<long long *>(base + o_off);
    pa.voff = reinterpret_cast<long long *>(base + o_voff);
    pa.Gin = G;
    pa.sigma = sigma;
    pa.U = U;
    pa.V = want_v ? V : nullptr;
    pa.lambda = lambda;
    pa.want_v = want_v ? 1 : 0;
    pa.ordering = prm.ordering;
    pa.sort = prm.sort ? 1 : 0;
    pa.max_sweeps = max_sweeps;
    pa.tol = prm.tol;
    pa.tthresh = prm.t_thresh;
    pa.status = reinterpret_cast<int *>(base + o_st);
    pa.sweeps = reinterpret_cast<int *>(base + o_sw);
    pa.code = reinterpret_cast<int *>(base + o_code);
    pa.maxt = reinterpret_cast<double *>(base + o_mt);
    pa.rot = reinterpret_cast<unsigned long long *>(base + o_rot);
    pa.skip = reinterpret_cast<unsigned long long *>(base + o_skip);
    pa.act = reinterpret_cast<unsigned long long *>(base + o_act);
    pa.mixed = prm.precision == HSVD_MIXED ? 1 : 0;
    pa.reorth_accept = prm.reorth_accept;
    pa.sweeps32 = reinterpret_cast<int *>(base + o_s32);
    pa.nsiters = reinterpret_cast<int *>(base + o_ni);
    pa.restart = reinterpret_cast<int *>(base + o_rs);
    pa.nsres = reinterpret_cast<double *>(base + o_nr);
    pa.slots = base + o_slots;
    if (prm.graph) {
        if (!ctx->cap) HSVD_TRY(hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
        if (!ctx->join) HSVD_TRY(hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming));
        hipStream_t q = ctx->cap;
        HSVD_TRY(hipEventRecord(ctx->join, st));
        HSVD_TRY(hipStreamWaitEvent(q, ctx->join, 0));
        HSVD_TRY(hipStreamBeginCapture(q, hipStreamCaptureModeThreadLocal));
        const hipError_t le = launch_batch_persist(q, pa, threads, wgs);
        hipGraph_t graph = nullptr;
        const hipError_t ee = hipStreamEndCapture(q, &graph);
        if (le != hipSuccess || ee != hipSuccess) {
            if (graph) hipGraphDestroy(graph);
            return HSVD_E_DEVICE;
        }
        hipGraphExec_t exec = nullptr;
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            hipGraphDestroy(graph);
            return HSVD_E_DEVICE;
        }
        const hipError_t ge = hipGraphLaunch(exec, q);
        hipError_t je = hipEventRecord(ctx->join, q);
        if (je == hipSuccess) je = hipStreamWaitEvent(st, ctx->join, 0);
        const hipError_t se = hipStreamSynchronize(st);
        hipGraphExecDestroy(exec);
        hipGraphDestroy(graph);
        if (ge != hipSuccess || je != hipSuccess || se != hipSuccess) return HSVD_E_DEVICE;
    } else {
        HSVD_TRY(launch_batch_persist(st, pa, threads, wgs));
    }
    std::vector<int> hs(batch), hsw(batch), hc(batch);
    std::vector<double> hm(batch);
    std::vector<unsigned long long> hr(batch), hk(batch), ha(batch);
    HSVD_TRY(hipMemcpyAsync(hs.data(), pa.status, sizeof(int) * batch, hipMemcpyDeviceToHost, st));
    HSVD_TRY(hipMemcpyAsync(hsw.data(), pa.sweeps, sizeof(int) * batch, hipMemcpyDeviceToHost, st));
    HSVD_TRY(hipMemcpyAsync(hc.data(), pa.code, sizeof(int) * batch, hipMemcpyDeviceToHost, st));
    HSVD_TRY(hipMemcpyAsync(hm.data(), pa.maxt, sizeof(double) * batch, hipMemcpyDeviceToHost, st));
    HSVD_TRY(hipMemcpyAsync(hr.data(), pa.rot, sizeof(unsigned long long) * batch, hipMemcpyDeviceToHost, st));
    HSVD_TRY(hipMemcpyAsync(hk.data(), pa.skip, sizeof(unsigned long long) * batch, hipMemcpyDeviceToHost, st));
    HSVD_TRY(hipMemcpyAsync(ha.data(), pa.act, sizeof(unsigned long long) * batch, hipMemcpyDeviceToHost, st));
    std::vector<int> h32(batch), hni(batch), hrs(batch);
    std::vector<double> hres(batch);
    if (pa.mixed) {
        HSVD_TRY(hipMemcpyAsync(h32.data(), pa.sweeps32, sizeof(int) * batch, hipMemcpyDeviceToHost, st));
        HSVD_TRY(hipMemcpyAsync(hni.data(), pa.nsiters, sizeof(int) * batch, hipMemcpyDeviceToHost, st));
        HSVD_TRY(hipMemcpyAsync(hrs.data(), pa.restart, sizeof(int) * batch, hipMemcpyDeviceToHost, st));
        HSVD_TRY(hipMemcpyAsync(hres.data(), pa.nsres, sizeof(double) * batch, hipMemcpyDeviceToHost, st));
    }
    HSVD_TRY(hipStreamSynchronize(st));
    const int b = block_width();
    for (int k : ids) {
        hsvd_info &pi = pinfo[k];
        const int r = (n[k] + 2 * b - 1) / (2 * b) * (2 * b), nb = r / b;
        pi.status = hs[k];
        pi.sweeps = hsw[k];
        pi.code = hc[k];
        pi.r = r;
        pi.block = b;
        pi.ldg = r;
        pi.max_t_last = hm[k];
        pi.rotations = (long long)hr[k];
        pi.skips = (long long)hk[k];
        pi.steps = (long long)hsw[k] * (prm.ordering == HSVD_ORD_MODMOD ? nb : nb - 1);
        pi.active_pairs = (long long)ha[k];
        if (pa.mixed) {
            pi.sweeps_fp32 = h32[k];
            pi.reorth_iters = hni[k];
            pi.fp64_restart = hrs[k];
            pi.reorth_resid = hres[k] <= 1.0 ? hres[k] : 0.0;
        }
    }
    return HSVD_OK;
}

extern "C" hsvd_status hsvd_solve_batched(hsvd_ctx *ctx, int batch, const int *n_in, const int *p_in,
                                          const long long *off_in, const long long *voff_in, const double *G,
                                          const hsvd_params *prm_in, double *sigma, double *U, double *V,
                                          double *lambda, hsvd_info *info)
{
    if (!ctx || batch < 0) return HSVD_E_INVAL;
    if (batch == 0) return HSVD_OK;
    if (!n_in || !p_in || !off_in || !voff_in || !G || !sigma) return HSVD_E_INVAL;
    hsvd_params prm;
    if (prm_in) prm = *prm_in;
    else hsvd_default_params(&prm);
    if (prm.precision != HSVD_FP64 && prm.precision != HSVD_MIXED) return HSVD_E_INVAL;
    const bool mixed = prm.precision == HSVD_MIXED;
    if (prm.ordering != HSVD_ORD_MODMOD && prm.ordering != HSVD_ORD_ROUNDROBIN) return HSVD_E_INVAL;
    if (prm.block != 0 && prm.block != block_width()) return HSVD_E_INVAL;
    if (prm.inner_sweeps < 0 || prm.inner_sweeps > 100) return HSVD_E_INVAL;
    if (prm.batch_mode < 0 || prm.batch_mode > 2) return HSVD_E_INVAL;
    const bool want_v = prm.want_v != 0;
    if (V && !want_v) return HSVD_E_INVAL;
    // the mixed path carries V through its FP32 phase even when it is not returned
    const bool acc_v = want_v || mixed;
    HSVD_TRY(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    // the per-problem metadata, device or host memory, to the host once: it
    // decides the groups and their launch shapes
    std::vector<int> n(batch), p(batch);
    std::vector<long long> off(batch), voff(batch);
    HSVD_TRY(hipMemcpyAsync(n.data(), n_in, sizeof(int) * batch, hipMemcpyDefault, st));
    HSVD_TRY(hipMemcpyAsync(p.data(), p_in, sizeof(int) * batch, hipMemcpyDefault, st));
    HSVD_TRY(hipMemcpyAsync(off.data(), off_in, sizeof(long long) * batch, hipMemcpyDefault, st));
    HSVD_TRY(hipMemcpyAsync(voff.data(), voff_in, sizeof(long long) * batch, hipMemcpyDefault, st));
    HSVD_TRY(hipStreamSynchronize(st));
    for (int k = 0; k < batch; ++k)
        if (n[k] < 1 || n[k] > 1024 || p[k] < 0 || p[k] > n[k] || off[k] < 0 || voff[k] < 0) return HSVD_E_INVAL;
    const int max_sweeps = prm.max_sweeps > 0 ? prm.max_sweeps : 100;
    const int b = block_width();
    hsvd_status s = ensure_events(ctx, 4 + 4 * 1024 / b);
    if (s != HSVD_OK) return s;
    hipEvent_t *ev = ctx->events.data();

    // FP64 block-oriented problems with n <= kPersistMaxOrder: one persistent
    // launch (batch_mode 0); the others grouped by bordered order r = n
    // rounded up to 2b, one sequence of launches per group
    std::vector<int> pers;
    std::vector<std::vector<int>> groups(1024 / (2 * b) + 1);
    // batch_mode 2: the schedule the autotuner chose for this precision, else
    // the persistent launch
    const int sched = prm.batch_mode == 2 ? std::max(0, ctx->batch_sched[mixed ? 1 : 0]) : prm.batch_mode;
    const bool persist_ok = prm.inner_sweeps == 0 && sched == 0;
    for (int k = 0; k < batch; ++k) {
        if (persist_ok && n[k] <= kPersistMaxOrder)
            pers.push_back(k);
        else
            groups[(n[k] + 2 * b - 1) / (2 * b)].push_back(k);
    }

    // per-problem results, filled group by group
    std::vector<hsvd_info> pinfo(batch);
    memset(pinfo.data(), 0, sizeof(hsvd_info) * batch);
    HSVD_TRY(hipEventRecord(ev[0], st));
    s = batch_persistent(ctx, st, pers, n.data(), p.data(), off.data(), voff.data(), G, prm, max_sweeps, want_v, sigma,
                         U, V, lambda, pinfo);
    if (s != HSVD_OK) return s;
    for (size_t gi = 1; gi < groups.size(); ++gi) {
        const std::vector<int> &ids = groups[gi];
        if (ids.empty()) continue;
        const int K = (int)ids.size();
        const int r = (int)gi * 2 * b, ldg = r, nb = r / b, pairs = nb / 2;
        const int steps_per_sweep = prm.ordering == HSVD_ORD_MODMOD ? nb : nb - 1;
        const size_t mat = (size_t)ldg * r, bb = (size_t)4 * b * b;
        // workspace of the group
        size_t o = 0;
        const size_t o_ids = take_bytes(o, sizeof(int) * K), o_n = take_bytes(o, sizeof(int) * K);
        const size_t o_p = take_bytes(o, sizeof(int) * K), o_done = take_bytes(o, sizeof(int) * K);
        const size_t o_stat = take_bytes(o, sizeof(int) * K), o_sw = take_bytes(o, sizeof(int) * K);
        const size_t o_off = take_bytes(o, sizeof(long long) * K), o_voff = take_bytes(o, sizeof(long long) * K);
        const size_t o_tol = take_bytes(o, sizeof(double) * K), o_tth = take_bytes(o, sizeof(double) * K);
        const size_t o_cnt = take_bytes(o, sizeof(int));
        const size_t o_G = take_bytes(o, sizeof(double) * mat * K);
        const size_t o_V = take_bytes(o, acc_v ? sizeof(double) * mat * K : 0);
        const size_t o_d = take_bytes(o, sizeof(double) * r * K), o_dt = take_bytes(o, sizeof(double) * r * K);
        const size_t o_rho = take_bytes(o, sizeof(int) * r * K), o_rt = take_bytes(o, sizeof(int) * r * K);
        const size_t o_C = take_bytes(o, sizeof(int) * pairs * K);
        const size_t o_nr = take_bytes(o, sizeof(unsigned) * pairs * K);
        const size_t o_ns = take_bytes(o, sizeof(unsigned) * pairs * K);
        const size_t o_na = take_bytes(o, sizeof(unsigned) * pairs * K);
        const size_t o_ntc = take_bytes(o, sizeof(unsigned) * pairs * K);
        const size_t o_mt = take_bytes(o, sizeof(double) * pairs * K);
        const size_t o_ctl = take_bytes(o, sizeof(Ctl) * K);
        const size_t o_S2 = take_bytes(o, sizeof(int4) * 2 * pairs);
        const size_t o_P = take_bytes(o, sizeof(double) * pairs * bb * K);
        const size_t o_W = take_bytes(o, sizeof(double) * pairs * bb * K);
        const size_t o_act = take_bytes(o, sizeof(unsigned long long) * pairs * K);
        // mixed: FP32 copies, the Newton-Schulz products and the per-problem
        // state (the FP32 partial Grams and W live in the FP64 ones' space)
        const size_t mx_mat = mixed ? mat * K : 0, mx_k = mixed ? (size_t)K : 0;
        const size_t o_G32 = take_bytes(o, sizeof(float) * mx_mat), o_V32 = take_bytes(o, sizeof(float) * mx_mat);
        const size_t o_T1 = take_bytes(o, sizeof(double) * mx_mat), o_T2 = take_bytes(o, sizeof(double) * mx_mat);
        const size_t o_d32 = take_bytes(o, sizeof(int) * mx_k), o_s32 = take_bytes(o, sizeof(int) * mx_k);
        const size_t o_pm = take_bytes(o, sizeof(double) * mx_k), o_pf = take_bytes(o, sizeof(double) * mx_k);
        const size_t o_t32 = take_bytes(o, sizeof(double) * mx_k), o_h32 = take_bytes(o, sizeof(double) * mx_k);
        const size_t o_ap = take_bytes(o, sizeof(int) * mx_k), o_nd = take_bytes(o, sizeof(int) * mx_k);
        const size_t o_np = take_bytes(o, sizeof(double) * mx_k);
        const size_t o_ni = take_bytes(o, sizeof(int) * mx_k), o_rs = take_bytes(o, sizeof(int) * mx_k);
        s = ensure_ws(ctx, o);
        if (s != HSVD_OK) return s;
        char *base = static_cast<char *>(ctx->ws);
        // per-problem metadata
        std::vector<int> hn(K), hp(K);
        std::vector<long long> hoff(K), hvoff(K);
        std::vector<double> htol(K), htth(K);
        for (int z = 0; z < K; ++z) {
            const int k = ids[z];
            hn[z] = n[k];
            hp[z] = p[k];
            hoff[z] = off[k];
            hvoff[z] = voff[k];
            htol[z] = prm.tol > 0.0 ? prm.tol : 1e-15 * n[k];
            htth[z] = prm.t_thresh > 0.0 ? prm.t_thresh : sqrt(htol[z]) / 2.0;
        }
        HSVD_TRY(hipMemcpyAsync(base + o_ids, ids.data(), sizeof(int) * K, hipMemcpyHostToDevice, st));
        HSVD_TRY(hipMemcpyAsync(base + o_n, hn.data(), sizeof(int) * K, hipMemcpyHostToDevice, st));
        HSVD_TRY(hipMemcpyAsync(base + o_p, hp.data(), sizeof(int) * K, hipMemcpyHostToDevice, st));
        HSVD_TRY(hipMemcpyAsync(base + o_off, hoff.data(), sizeof(long long) * K, hipMemcpyHostToDevice, st));
        HSVD_TRY(hipMemcpyAsync(base + o_voff, hvoff.data(), sizeof(long long) * K, hipMemcpyHostToDevice, st));
        HSVD_TRY(hipMemcpyAsync(base + o_tol, htol.data(), sizeof(double) * K, hipMemcpyHostToDevice, st));
        HSVD_TRY(hipMemcpyAsync(base + o_tth, htth.data(), sizeof(double) * K, hipMemcpyHostToDevice, st));
        HSVD_TRY(hipStreamSynchronize(st));

        BatchGroup g;
        g.nprob = K;
        g.r = r;
        g.ldg = ldg;
        g.pairs = pairs;
        g.max_sweeps = max_sweeps;
        g.ids = reinterpret_cast<int *>(base + o_ids);
        g.n = reinterpret_cast<int *>(base + o_n);
        g.p = reinterpret_cast<int *>(base + o_p);
        g.off = reinterpret_cast<long long *>(base + o_off);
        g.voff = reinterpret_cast<long long *>(base + o_voff);
        g.tol = reinterpret_cast<double *>(base + o_tol);
        g.tth = reinterpret_cast<double *>(base + o_tth);
        g.done = reinterpret_cast<int *>(base + o_done);
        g.status = reinterpret_cast<int *>(base + o_stat);
        g.sweeps = reinterpret_cast<int *>(base + o_sw);
        g.active_count = reinterpret_cast<int *>(base + o_cnt);
        g.G = reinterpret_cast<double *>(base + o_G);
        g.V = acc_v ? reinterpret_cast<double *>(base + o_V) : nullptr;
        g.d = reinterpret_cast<double *>(base + o_d);
        g.dtmp = reinterpret_cast<double *>(base + o_dt);
        g.rho = reinterpret_cast<int *>(base + o_rho);
        g.rtmp = reinterpret_cast<int *>(base + o_rt);
        g.C = reinterpret_cast<int *>(base + o_C);
        g.nrot = reinterpret_cast<unsigned *>(base + o_nr);
        g.nskip = reinterpret_cast<unsigned *>(base + o_ns);
        g.nact = reinterpret_cast<unsigned *>(base + o_na);
        g.ntc = reinterpret_cast<unsigned *>(base + o_ntc);
        g.maxt = reinterpret_cast<double *>(base + o_mt);
        g.ctl = reinterpret_cast<Ctl *>(base + o_ctl);
        int4 *S2 = reinterpret_cast<int4 *>(base + o_S2);

        HSVD_TRY(launch_batch_setup(st, g, G, acc_v));
        HSVD_TRY(launch_block_stepper_init(st, S2, nb));
        if (prm.sort) HSVD_TRY(launch_batch_sort(st, g));

        BlockArgs ba;
        ba.G = g.G;
        ba.V = g.V;
        ba.ldg = ldg;
        ba.r = r;
        ba.p = 0;
        ba.nb = nb;
        ba.rho = g.rho;
        ba.ordering = prm.ordering;
        ba.partial = reinterpret_cast<double *>(base + o_P);
        ba.splits = 1;
        ba.rows_per_split = ldg;
        ba.W = reinterpret_cast<double *>(base + o_W);
        ba.active = reinterpret_cast<unsigned long long *>(base + o_act);
        ba.C = g.C;
        ba.nrot = g.nrot;
        ba.nskip = g.nskip;
        ba.nact = g.nact;
        ba.ntc = g.ntc;
        ba.maxt = g.maxt;
        ba.ctl = g.ctl;
        ba.tol = 0.0;
        ba.tthresh = 0.0;
        ba.inner_sweeps = prm.inner_sweeps;
        ba.nprob = K;
        ba.done = g.done;
        ba.pvec = g.p;
        ba.tolvec = g.tol;
        ba.tthvec = g.tth;
        long long gstep = 0;
        int gsweeps = 0;
        int *host_active = &ctx->host_ctl->code;  // pinned scratch for the count of running problems
        if (mixed) {
            BatchMixed m;
            m.G32 = reinterpret_cast<float *>(base + o_G32);
            m.V32 = reinterpret_cast<float *>(base + o_V32);
            m.T1 = reinterpret_cast<double *>(base + o_T1);
            m.T2 = reinterpret_cast<double *>(base + o_T2);
            m.done32 = reinterpret_cast<int *>(base + o_d32);
            m.sweeps32 = reinterpret_cast<int *>(base + o_s32);
            m.prev_maxt = reinterpret_cast<double *>(base + o_pm);
            m.prev_frac = reinterpret_cast<double *>(base + o_pf);
            m.tol32 = reinterpret_cast<double *>(base + o_t32);
            m.tth32 = reinterpret_cast<double *>(base + o_h32);
            m.apply = reinterpret_cast<int *>(base + o_ap);
            m.nsdone = reinterpret_cast<int *>(base + o_nd);
            m.nsprev = reinterpret_cast<double *>(base + o_np);
            m.nsiters = reinterpret_cast<int *>(base + o_ni);
            m.restart = reinterpret_cast<int *>(base + o_rs);
            m.accept = prm.reorth_accept;
            int sw32 = 0;
            s = batch_mixed_phase(ctx, st, g, m, ba, S2, pairs, steps_per_sweep, max_sweeps, prm.sort != 0, gstep,
                                  host_active, sw32, G);
            if (s != HSVD_OK) return s;
            // per-problem FP32 sweeps, corrections, final residuals, restarts
            std::vector<int> h32(K), hni(K), hrs(K);
            std::vector<double> hres(K);
            HSVD_TRY(hipMemcpyAsync(h32.data(), m.sweeps32, sizeof(int) * K, hipMemcpyDeviceToHost, st));
            HSVD_TRY(hipMemcpyAsync(hni.data(), m.nsiters, sizeof(int) * K, hipMemcpyDeviceToHost, st));
            HSVD_TRY(hipMemcpyAsync(hrs.data(), m.restart, sizeof(int) * K, hipMemcpyDeviceToHost, st));
            HSVD_TRY(hipMemcpyAsync(hres.data(), m.nsprev, sizeof(double) * K, hipMemcpyDeviceToHost, st));
            HSVD_TRY(hipStreamSynchronize(st));
            for (int z = 0; z < K; ++z) {
                hsvd_info &pi = pinfo[ids[z]];
                pi.sweeps_fp32 = h32[z];
                pi.reorth_iters = hni[z];
                pi.fp64_restart = hrs[z];
                pi.reorth_resid = hres[z] <= 1.0 ? hres[z] : 0.0;
            }
        }
        // one sweep: the outer steps, the kept diagonal, the sort, the stop rule
        auto enqueue_sweep = [&](hipStream_t q, bool timed) -> hipError_t {
            for (int k = 0; k < steps_per_sweep; ++k, ++gstep) {
                ba.step = k;
                ba.S_in = S2 + (gstep & 1) * pairs;
                ba.S_out = S2 + ((gstep + 1) & 1) * pairs;
                hipEvent_t *e = ev + 4 + 4 * k;
                hipError_t er;
                if (timed && (er = hipEventRecord(e[0], q)) != hipSuccess) return er;
                if ((er = launch_block_gram<double>(q, ba)) != hipSuccess) return er;
                if (timed && (er = hipEventRecord(e[1], q)) != hipSuccess) return er;
                if ((er = launch_block_inner<double>(q, ba)) != hipSuccess) return er;
                if (timed && (er = hipEventRecord(e[2], q)) != hipSuccess) return er;
                if ((er = launch_block_update<double>(q, ba)) != hipSuccess) return er;
                if (timed && (er = hipEventRecord(e[3], q)) != hipSuccess) return er;
            }
            hipError_t er;
            if ((er = launch_batch_colnorm(q, g, false)) != hipSuccess) return er;
            if (prm.sort && (er = launch_batch_sort(q, g)) != hipSuccess) return er;
            if ((er = launch_batch_reduce_decide(q, g)) != hipSuccess) return er;
            return hipMemcpyAsync(host_active, g.active_count, sizeof(int), hipMemcpyDeviceToHost, q);
        };
        hipGraphExec_t exec = nullptr;
        hipGraph_t graph = nullptr;
        hipStream_t q = st;
        if (prm.graph) {
            // steps_per_sweep is even for the modified modulus ordering, so the
            // stepper's double buffer is in the same phase at every sweep and
            // one captured sweep serves them all (round-robin keeps no state)
            if (!ctx->cap) HSVD_TRY(hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
            if (!ctx->join) HSVD_TRY(hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming));
            q = ctx->cap;
            HSVD_TRY(hipEventRecord(ctx->join, st));
            HSVD_TRY(hipStreamWaitEvent(q, ctx->join, 0));
            HSVD_TRY(hipStreamBeginCapture(q, hipStreamCaptureModeThreadLocal));
            const long long g0 = gstep;
            const hipError_t ce = enqueue_sweep(q, false);
            gstep = g0;
            hipError_t ee = hipStreamEndCapture(q, &graph);
            if (ce != hipSuccess || ee != hipSuccess) {
                if (graph) hipGraphDestroy(graph);
                return HSVD_E_DEVICE;
            }
            if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
                hipGraphDestroy(graph);
                return HSVD_E_DEVICE;
            }
        }
        for (int sw = 0; sw < max_sweeps; ++sw) {
            if (prm.graph) {
                HSVD_TRY(hipGraphLaunch(exec, q));
                gstep += steps_per_sweep;
            } else {
                HSVD_TRY(enqueue_sweep(q, false));
            }
            HSVD_TRY(hipStreamSynchronize(q));
            const int active = *host_active;
            ++gsweeps;
            if (active == 0) break;
        }
        if (prm.graph) {
            hipGraphExecDestroy(exec);
            hipGraphDestroy(graph);
            HSVD_TRY(hipEventRecord(ctx->join, q));
            HSVD_TRY(hipStreamWaitEvent(st, ctx->join, 0));
        }
        HSVD_TRY(launch_batch_finalize(st, g, sigma, U, want_v ? V : nullptr, lambda));
        std::vector<int> hs(K), hsw(K);
        std::vector<Ctl> hctl(K);
        HSVD_TRY(hipMemcpyAsync(hs.data(), g.status, sizeof(int) * K, hipMemcpyDeviceToHost, st));
        HSVD_TRY(hipMemcpyAsync(hsw.data(), g.sweeps, sizeof(int) * K, hipMemcpyDeviceToHost, st));
        HSVD_TRY(hipMemcpyAsync(hctl.data(), g.ctl, sizeof(Ctl) * K, hipMemcpyDeviceToHost, st));
        HSVD_TRY(hipStreamSynchronize(st));
        for (int z = 0; z < K; ++z) {
            hsvd_info &pi = pinfo[ids[z]];
            pi.status = hs[z];
            pi.sweeps = hsw[z];
            pi.code = hctl[z].code;
            pi.r = r;
            pi.block = b;
            pi.ldg = ldg;
            pi.max_t_last = hctl[z].maxt;
            pi.rotations = (long long)hctl[z].rot;
            pi.skips = (long long)hctl[z].skip;
            pi.steps = (long long)hsw[z] * steps_per_sweep;
            pi.active_pairs = (long long)hctl[z].act;
        }
        (void)gsweeps;
    }
    HSVD_TRY(hipEventRecord(ev[1], st));
    HSVD_TRY(hipStreamSynchronize(st));
    float ms = 0.f;
    HSVD_TRY(hipEventElapsedTime(&ms, ev[0], ev[1]));
    hsvd_status result = HSVD_OK;
    for (int k = 0; k < batch; ++k) {
        pinfo[k].ms_total = ms;
        if (result == HSVD_OK && pinfo[k].status != HSVD_OK) result = (hsvd_status)pinfo[k].status;
    }
    if (info) {
        HSVD_TRY(hipMemcpyAsync(info, pinfo.data(), sizeof(hsvd_info) * batch, hipMemcpyDefault, st));
        HSVD_TRY(hipStreamSynchronize(st));
    }
    return result;
}

extern "C" {

static hsvd_status pair_params_common(hsvd_ctx *ctx, long long m, const double *aii, const double *ajj,
                                      const double *aij, const int *hyp, double tol, double t_thresh, int *skip,
                                      double *t, double *c, int *status, int *code, bool fast)
{
    if (!ctx || m < 0) return HSVD_E_INVAL;
    if (m > 0 && (!aii || !ajj || !aij || !hyp || !skip || !t || !c || !status || !code))
        return HSVD_E_INVAL;
    HSVD_TRY(hipSetDevice(ctx->device));
    HSVD_TRY(launch_pair_params(ctx->stream, m, aii, ajj, aij, hyp, tol, t_thresh, skip, t, c, status,
                                code, fast));
    HSVD_TRY(hipStreamSynchronize(ctx->stream));
    return HSVD_OK;
}

hsvd_status hsvd_pair_params(hsvd_ctx *ctx, long long m, const double *aii, const double *ajj,
                             const double *aij, const int *hyp, double tol, double t_thresh, int *skip,
                             double *t, double *c, int *status, int *code)
{
    return pair_params_common(ctx, m, aii, ajj, aij, hyp, tol, t_thresh, skip, t, c, status, code, false);
}

hsvd_status hsvd_block_pair_params(hsvd_ctx *ctx, long long m, const double *aii, const double *ajj,
                                   const double *aij, const int *hyp, double tol, double t_thresh, int *skip,
                                   double *t, double *c, int *status, int *code)
{
    return pair_params_common(ctx, m, aii, ajj, aij, hyp, tol, t_thresh, skip, t, c, status, code, true);
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
    if (!ctx || (b != block_width() && b != kWideB) || r < 2 * b || r % (2 * b) || r > kMaxOrder || steps < 0 ||
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
