// Block-column one-sided Jacobi HSVD kernels for gfx950 (FP64 or FP32 MFMA).
//
// Positions are split into nb = r / b blocks of b consecutive positions; a
// parallel step pairs blocks (I, J) by the outer ordering (modified modulus
// or round-robin over nb), as in the block-oriented algorithm of Sec. 5.  For
// each block pair the 2b columns G_P = [G_I G_J] (gathered through rho) are
// processed in three launches:
//
//   block_gram_kernel    A_P = G_P^T G_P on 16x16x4 MFMA, split over row
//                        ranges; partial Grams summed in a fixed order.
//   block_inner_*_kernel one workgroup per pair: rotations of the pointwise
//                        method (eqs. 2.2-2.5, in the short-chain form of
//                        rotation_params_fast) applied two-sided to A_P and to
//                        the columns of the accumulated W, in a parallel inner
//                        ordering (circle kernel: A_P and W in LDS; cross
//                        kernel: both in registers).  With V carried, extra
//                        workgroups of the cross kernel apply the previous
//                        step's W to V.
//   block_update_kernel  [G_P | V_P] <- [G_P | V_P] W on MFMA, row tiles
//                        (G alone when V's half runs in the inner launch).
//
// Inner ordering: in the first outer step of a sweep every pair of the 2b
// columns once (circle method over 2b indices, 2b - 1 inner steps); in the
// other outer steps only the b^2 cross pairs (x, b + ((x + u) mod b)),
// b inner steps.
//
// The kernels are templated on the storage type T of G, V, the partial Grams
// and W: double for the FP64 path, float for the FP32 sweeps of the mixed
// path (FP32 MFMA with FP32 accumulation).  The partial Grams are summed in
// FP64.  The circle kernel holds A_P and W in FP64 and rounds W to T on
// output; the cross kernel holds its blocks of A_P and W in T and computes
// each rotation's parameters in FP64 from the T-held pivots, applying them in
// T.
//
// The bodies of the Gram, the inner solves and the update are device
// functions in block_device.h (shared with the persistent batched kernel);
// the kernels here bind a launch's block indices to them.
#include "block_device.h"

namespace hsvd {

// V update of the previous outer step, run by extra workgroups of an inner
// launch (defined with the update kernel).
template <typename T>
__device__ void v_update_role(const BlockArgsT<T> &a, int role);

// ---------------------------------------------------------------------------
// Per-launch kernels: one workgroup per block pair (and row split)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void block_gram_kernel(BlockArgsT<T> a)
{
    __shared__ T red[kGramRed];
    if (!bind_problem(a)) return;
    gram_pair<T>(a, blockIdx.x, blockIdx.y, red);
}

template <typename T>
__global__ __launch_bounds__(1024) void block_inner_circle_kernel(BlockArgsT<T> a)
{
    __shared__ CircleLds L;
    if (!bind_problem(a)) return;
    inner_circle_pair<T, 1024>(a, blockIdx.x, L);
}

// With NT = b^2 (single solves) the workgroups after the block pairs' own
// apply the previous outer step's W to V (v_update_role).
template <typename T, int NT>
__global__ __launch_bounds__(NT) void block_inner_cross_kernel(BlockArgsT<T> a)
{
    __shared__ CrossLds<T> L;
    if constexpr (NT == kB * kB) {
        if ((int)blockIdx.x >= a.nb / 2) {
            v_update_role(a, (int)blockIdx.x - a.nb / 2);
            return;
        }
    }
    if (!bind_problem(a)) return;
    inner_cross_pair<T, NT>(a, blockIdx.x, L);
}

// launches).
// Tiles of the update kernel: rows [t * rows, (t + 1) * rows) of G for
// t < tiles_g, of V after that; a.tile0 shifts the tile index (G-only and
// V-only launches).  The tile runs along blockIdx.x and the block pair along
// blockIdx.y: consecutive workgroups go to the 8 XCDs in turn, so every XCD
// takes an equal share of every pair's rows.  With the pair along x, an XCD
// took whole pairs (those congruent mod 8), and since pairs without a rotation
// or with few touched columns do little, the busiest XCD set the launch time
// (FP32 update at n = 4096: 29.7 -> 25.3 us per launch, bit-identical).
template <typename T>
__global__ __launch_bounds__(256, UpdCfg<T>::min_blocks) void block_update_kernel(BlockArgsT<T> a)
{
    constexpr int kRows = UpdCfg<T>::rows, kUpdLd = UpdCfg<T>::ld;
    __shared__ T Wl[kB2 * kUpdLd];
    __shared__ int cols[kB2];
    __shared__ int tl[kB2];
    const int k = blockIdx.y;
    const int tiles_g = (a.ldg + kRows - 1) / kRows;
    const int t = blockIdx.x + a.tile0;
    if (t == 0 && blockIdx.z == 0 && threadIdx.x == 0 && a.ordering == HSVD_ORD_MODMOD)
        a.S_out[k] = modmod_next(a.S_in[k], a.nb);
    if (!bind_problem(a)) return;
    const unsigned long long mask = a.active[k];
    if (!mask) return;  // no rotation in this pair: W = I
    T *__restrict__ M = t < tiles_g ? a.G : a.V;
    const int row_base = (t < tiles_g ? t : t - tiles_g) * kRows;
    const int nstrips = min(kRows, a.ldg - row_base) / 16;
    update_rows<T, 256, UpdCfg<T>::w_lds, true, kUpdLd>(a, k, M, row_base, nstrips, mask, Wl, cols, tl);
}

// V update of the previous outer step inside an inner-solve launch: workgroup
// `role` (after the block pairs' own workgroups) takes rows [tile * a.vrows,
// ...) of V for block pair role / tiles.  The inner solve holds only one
// workgroup per block pair, most CUs are free meanwhile, and the next step's
// Gram needs G alone, so V's half of the update runs here instead of after
// the inner solve.  1024 threads: W from LDS (the 64 W operands do not fit
// the register budget of a 1024-thread workgroup), prefetch for FP32 only.
template <typename T>
__device__ void v_update_role(const BlockArgsT<T> &a, int role)
{
    constexpr int kLdV = sizeof(T) == 8 ? kB2 + 8 : kB2 + 16;
    __shared__ T Wl[kB2 * kLdV];
    __shared__ int cols[kB2];
    __shared__ int tl[kB2];
    const int tiles = (a.ldg + a.vrows - 1) / a.vrows;
    const int k = role / tiles, tile = role - k * tiles;
    BlockArgsT<T> v = a;
    v.W = a.W_prev;
    v.active = a.active_prev;
    v.S_in = a.S_prev;
    v.step = a.step_prev;
    const unsigned long long mask = v.active[k];
    if (!mask) return;
    const int row_base = tile * a.vrows;
    const int nstrips = min(a.vrows, a.ldg - row_base) / 16;
    update_rows<T, 1024, true, true, kLdV>(v, k, a.V, row_base, nstrips, mask, Wl, cols, tl);
}

// Outer stepper start (nb/2 slots, antidiagonal over blocks).
__global__ void block_stepper_init_kernel(int4 *S, int nb)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nb / 2) S[k] = modmod_start(k, nb);
}

// d[pos] = ||G[:, rho[pos]]||^2, one workgroup per position.
template <typename T>
__global__ __launch_bounds__(256) void colnorm_pos_kernel(const T *__restrict__ G, int ldg,
                                                          const int *__restrict__ rho,
                                                          double *__restrict__ d)
{
    __shared__ double sh[4];
    const int q = blockIdx.x;
    const T *gc = G + (size_t)rho[q] * ldg;
    double s = 0.0;
    for (int row = threadIdx.x; row < ldg; row += 256) {
        const double x = (double)gc[row];
        s = fma(x, x, s);
    }
    s = block_sum<256>(s, sh);
    if (threadIdx.x == 0) d[q] = s;
}

// Diagnostic: positions (i, j), i < j, of every inner pair of outer step
// `step` (sweep-relative), in the order block pair, inner step, slot.
__global__ void block_trace_kernel(int ordering, int r, int b, int step, const int4 *__restrict__ S,
                                   int *__restrict__ out)
{
    const int nb = r / b;
    const int k = blockIdx.x;
    if (k >= nb / 2) return;
    int I, J;
    if (ordering == HSVD_ORD_MODMOD) {
        I = S[k].z;
        J = S[k].w;
    } else {
        const int2 pr = roundrobin_pair(k, nb, step);
        I = pr.x;
        J = pr.y;
    }
    const bool first = step == 0;
    const int inner = first ? 2 * b - 1 : b;
    const int per = inner * b;
    for (int it = threadIdx.x; it < per; it += blockDim.x) {
        const int u = it / b, q = it % b;
        const int2 xy = block_inner_pair(q, u, first, b);
        const int pa = xy.x < b ? I * b + xy.x : J * b + xy.x - b;
        const int pb = xy.y < b ? I * b + xy.y : J * b + xy.y - b;
        int *o = out + ((size_t)k * per + it) * 2;
        o[0] = min(pa, pb);
        o[1] = max(pa, pb);
    }
}

__global__ void block_trace_advance_kernel(int4 *S, int nb)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nb / 2) S[k] = modmod_next(S[k], nb);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
int block_width() { return kB; }

hipError_t launch_block_stepper_init(hipStream_t st, int4 *S, int nb)
{
    block_stepper_init_kernel<<<(nb / 2 + 255) / 256, 256, 0, st>>>(S, nb);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_block_gram(hipStream_t st, const BlockArgsT<T> &a)
{
    block_gram_kernel<T><<<dim3(a.nb / 2, a.splits, a.nprob), 256, 0, st>>>(a);
    return hipGetLastError();
}

// Rows of V per role workgroup: the V update of one step spread over the CUs
// that the inner solves leave free (as many tiles per pair as fit, but at
// least 256 rows -- a 16-row strip per wave -- per tile), in whole 16-row
// strips so that the tiles of a pair come out nearly equal (the launch waits
// for the largest).
int v_update_role_rows(int pairs, int ldg, int cus, bool fp64)
{
    const int free_cus = cus > pairs ? cus - pairs : 1;
    // FP64: as many tiles again as there are CUs (the role workgroups queue
    // behind the first ones; shorter tiles balance better: FP64 inner launch
    // at n = 4096 50.6 -> 46.5 us, whole FP64 solve 220 -> 211 ms).  FP32:
    // one round on the free CUs (the same change made the FP32 launch slower,
    // 34.1 -> 36.6 us).
    int tiles = fp64 ? (free_cus + cus) / pairs : free_cus / pairs;
    if (tiles > ldg / 256) tiles = ldg / 256;
    if (tiles < 1) tiles = 1;
    int rows = (ldg + tiles - 1) / tiles;
    rows = (rows + 15) / 16 * 16;
    return rows < ldg ? rows : ldg;
}

int v_update_role_wgs(int pairs, int ldg, int vrows) { return pairs * ((ldg + vrows - 1) / vrows); }

template <typename T>
hipError_t launch_block_inner(hipStream_t st, const BlockArgsT<T> &a)
{
    // only the cross steps carry V-update workgroups (the first step of a
    // sweep has no previous step in it; the full-block method updates V in
    // its update launches)
    if (a.step == 0 || a.inner_sweeps > 0) {
        if (a.vprev_wgs > 0) return hipErrorInvalidValue;
        block_inner_circle_kernel<T><<<dim3(a.nb / 2, 1, a.nprob), 1024, 0, st>>>(a);
        return hipGetLastError();
    }
    if (a.vprev_wgs > 0 && a.nprob > 1) return hipErrorInvalidValue;
    if (a.nprob > 1) {
        // batched: throughput over latency -- 256 threads per block pair, four
        // pairs per CU, each thread four blocks of A_P
        block_inner_cross_kernel<T, 256><<<dim3(a.nb / 2, 1, a.nprob), 256, 0, st>>>(a);
    } else {
        block_inner_cross_kernel<T, kB * kB><<<dim3(a.nb / 2 + a.vprev_wgs, 1, a.nprob), kB * kB, 0, st>>>(a);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_block_update(hipStream_t st, const BlockArgsT<T> &a, int which)
{
    const int tiles_g = (a.ldg + UpdCfg<T>::rows - 1) / UpdCfg<T>::rows;
    BlockArgsT<T> b = a;
    int tiles = tiles_g * (a.V ? 2 : 1);
    b.tile0 = 0;
    if (which == UPD_G) {
        tiles = tiles_g;
    } else if (which == UPD_V) {
        if (!a.V) return hipSuccess;
        tiles = tiles_g;
        b.tile0 = tiles_g;
    }
    block_update_kernel<T><<<dim3(tiles, a.nb / 2, a.nprob), 256, 0, st>>>(b);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_colnorm_pos(hipStream_t st, const T *G, int ldg, const int *rho, double *d, int r)
{
    colnorm_pos_kernel<T><<<r, 256, 0, st>>>(G, ldg, rho, d);
    return hipGetLastError();
}

template hipError_t launch_block_gram<double>(hipStream_t, const BlockArgsT<double> &);
template hipError_t launch_block_gram<float>(hipStream_t, const BlockArgsT<float> &);
template hipError_t launch_block_inner<double>(hipStream_t, const BlockArgsT<double> &);
template hipError_t launch_block_inner<float>(hipStream_t, const BlockArgsT<float> &);
template hipError_t launch_block_update<double>(hipStream_t, const BlockArgsT<double> &, int);
template hipError_t launch_block_update<float>(hipStream_t, const BlockArgsT<float> &, int);
template hipError_t launch_colnorm_pos<double>(hipStream_t, const double *, int, const int *, double *, int);
template hipError_t launch_colnorm_pos<float>(hipStream_t, const float *, int, const int *, double *, int);

hipError_t launch_block_trace(hipStream_t st, int ordering, int r, int b, int step, int4 *S, int *out,
                              bool advance)
{
    block_trace_kernel<<<r / b / 2, 256, 0, st>>>(ordering, r, b, step, S, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !advance) return e;
    block_trace_advance_kernel<<<(r / b / 2 + 255) / 256, 256, 0, st>>>(S, r / b);
    return hipGetLastError();
}

}  // namespace hsvd
