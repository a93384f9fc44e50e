// Block-column one-sided Jacobi HSVD kernels for gfx950 (FP64 MFMA).
//
// Positions are split into nb = r / b blocks of b consecutive positions; a
// parallel step pairs blocks (I, J) by the outer ordering (modified modulus
// or round-robin over nb), as in the block-oriented algorithm of Sec. 5.  For
// each block pair the 2b columns G_P = [G_I G_J] (gathered through rho) are
// processed in three launches:
//
//   block_gram_kernel    A_P = G_P^T G_P on v_mfma_f64_16x16x4f64, split over
//                        row ranges; partial Grams summed in a fixed order.
//   block_inner_kernel   one workgroup per pair: A_P and the accumulated
//                        transformation W in LDS; rotations of the pointwise
//                        method (eqs. 2.2-2.5, the same parameter routine as the
//                        pairwise path) applied two-sided to A_P and to the
//                        columns of W, in a parallel inner ordering.
//   block_update_kernel  [G_P | V_P] <- [G_P | V_P] W on MFMA, row tiles.
//
// Inner ordering: in the first outer step of a sweep every pair of the 2b
// columns once (circle method over 2b indices, 2b - 1 inner steps); in the
// other outer steps only the b^2 cross pairs (x, b + ((x + u) mod b)),
// b inner steps.
#include "internal.h"

namespace hsvd {

typedef double d4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64 lane layout (wave64): operand A element (i, k) and
// operand B element (k, j) sit in lane i + 16k resp. j + 16k; accumulator
// register v of lane l holds D(l/16 + 4v, l%16).

constexpr int kB = 32;        // block width b
constexpr int kB2 = 2 * kB;   // columns of a block pair
constexpr int kLd = kB2 + 1;  // LDS row stride (doubles)

__device__ __forceinline__ int2 outer_pair(const BlockArgs &a, int k)
{
    if (a.ordering == HSVD_ORD_MODMOD) {
        const int4 s = a.S_in[k];
        return make_int2(s.z, s.w);
    }
    return roundrobin_pair(k, a.nb, a.step);
}

__device__ __forceinline__ int local_pos(int x, int I, int J)
{
    return x < kB ? I * kB + x : J * kB + (x - kB);
}

// ---------------------------------------------------------------------------
// Gram: partial[k][split] = G_P(rows of split)^T G_P(rows of split)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void block_gram_kernel(BlockArgs a)
{
    __shared__ double T[kB2 * kLd];
    __shared__ int cols[kB2];
    const int k = blockIdx.x, split = blockIdx.y;
    const int2 IJ = outer_pair(a, k);
    if (threadIdx.x < kB2) cols[threadIdx.x] = a.rho[local_pos(threadIdx.x, IJ.x, IJ.y)];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row_begin = split * a.rows_per_split;
    const int row_end = min(a.ldg, row_begin + a.rows_per_split);
    d4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
    for (int row0 = row_begin; row0 < row_end; row0 += 64) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int idx = threadIdx.x + 256 * e;
            const int c = idx >> 6, rr = idx & 63;
            T[c * kLd + rr] = a.G[(size_t)cols[c] * a.ldg + row0 + rr];
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < 16; ++kk) {
            const int rr = kk * 4 + (lane >> 4);
            const double av = T[(wave * 16 + (lane & 15)) * kLd + rr];
#pragma unroll
            for (int yt = 0; yt < 4; ++yt) {
                const double bv = T[(yt * 16 + (lane & 15)) * kLd + rr];
                acc[yt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[yt], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    double *out = a.partial + ((size_t)k * a.splits + split) * (kB2 * kB2);
#pragma unroll
    for (int yt = 0; yt < 4; ++yt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int x = wave * 16 + (lane >> 4) + 4 * v;
            const int y = yt * 16 + (lane & 15);
            out[x * kB2 + y] = acc[yt][v];
        }
}

// ---------------------------------------------------------------------------
// Inner solve of one block pair.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void block_inner_kernel(BlockArgs a)
{
    __shared__ double A[kB2 * kLd];
    __shared__ double Wl[kB2 * kLd];
    __shared__ double pt[kB], pc[kB], pht[kB];
    __shared__ int px[kB], py[kB], prot[kB];
    __shared__ int s_code, s_rot, s_skip;
    const int k = blockIdx.x;
    const int2 IJ = outer_pair(a, k);
    const double *P = a.partial + (size_t)k * a.splits * (kB2 * kB2);
    for (int idx = threadIdx.x; idx < kB2 * kB2; idx += 256) {
        double s = P[idx];
        for (int sp = 1; sp < a.splits; ++sp) s += P[(size_t)sp * (kB2 * kB2) + idx];
        const int x = idx / kB2, y = idx % kB2;
        A[x * kLd + y] = s;
        Wl[x * kLd + y] = x == y ? 1.0 : 0.0;
    }
    if (threadIdx.x == 0) {
        s_code = 0;
        s_rot = 0;
        s_skip = 0;
    }
    __syncthreads();

    const bool first = a.step == 0;
    const int inner_steps = first ? kB2 - 1 : kB;
    int code = 0, nrot = 0, nskip = 0, rank = 0;
    for (int u = 0; u < inner_steps; ++u) {
        if (threadIdx.x < kB) {
            const int q = threadIdx.x;
            const int2 xy = block_inner_pair(q, u, first, kB);
            const int x = xy.x, y = xy.y;
            const double axx = A[x * kLd + x], ayy = A[y * kLd + y], axy = A[x * kLd + y];
            double t = 0.0, c = 1.0;
            int rot = 0;
            if (rel_orthogonal(axx, ayy, axy, a.tol)) {
                ++nskip;
            } else {
                const int px_ = local_pos(x, IJ.x, IJ.y), py_ = local_pos(y, IJ.x, IJ.y);
                const int hyp = ((px_ < a.p) == (py_ < a.p)) ? -1 : 1;
                if (rotation_params(axx, ayy, axy, hyp, t, c)) {
                    rank = 1;
                    t = 0.0;
                    c = 1.0;
                } else {
                    rot = 1;
                    ++nrot;
                    code |= rotation_code(t, a.tthresh);
                    pht[q] = hyp < 0 ? -t : t;
                }
            }
            if (!rot) pht[q] = 0.0;
            pt[q] = t;
            pc[q] = c;
            px[q] = x;
            py[q] = y;
            prot[q] = rot;
        }
        __syncthreads();
        // A <- R^T A R on the 2x2 blocks (k1 <= k2), mirrored to keep A symmetric.
        for (int blk = threadIdx.x; blk < kB * kB; blk += 256) {
            const int k1 = blk / kB, k2 = blk % kB;
            if (k1 > k2) continue;
            const int x1 = px[k1], y1 = py[k1], x2 = px[k2], y2 = py[k2];
            const double t1 = pt[k1], c1 = pc[k1], h1 = pht[k1];
            const double t2 = pt[k2], c2 = pc[k2], h2 = pht[k2];
            double e00 = A[x1 * kLd + x2], e01 = A[x1 * kLd + y2];
            double e10 = A[y1 * kLd + x2], e11 = A[y1 * kLd + y2];
            // columns (x2, y2)
            double f00 = fma(h2, e01, e00) * c2, f01 = fma(t2, e00, e01) * c2;
            double f10 = fma(h2, e11, e10) * c2, f11 = fma(t2, e10, e11) * c2;
            // rows (x1, y1)
            e00 = fma(h1, f10, f00) * c1;
            e10 = fma(t1, f00, f10) * c1;
            e01 = fma(h1, f11, f01) * c1;
            e11 = fma(t1, f01, f11) * c1;
            if (k1 == k2) {
                if (prot[k1]) {
                    e01 = 0.0;
                    e10 = 0.0;
                }
                A[x1 * kLd + x1] = e00;
                A[y1 * kLd + y1] = e11;
                A[x1 * kLd + y1] = e01;
                A[y1 * kLd + x1] = e01;
            } else {
                A[x1 * kLd + x2] = e00;
                A[x1 * kLd + y2] = e01;
                A[y1 * kLd + x2] = e10;
                A[y1 * kLd + y2] = e11;
                A[x2 * kLd + x1] = e00;
                A[y2 * kLd + x1] = e01;
                A[x2 * kLd + y1] = e10;
                A[y2 * kLd + y1] = e11;
            }
        }
        // W <- W R on the columns of each pair.
        for (int it = threadIdx.x; it < kB2 * kB; it += 256) {
            const int q = it / kB2, w = it % kB2;
            if (!prot[q]) continue;
            const int x = px[q], y = py[q];
            const double wx = Wl[w * kLd + x], wy = Wl[w * kLd + y];
            Wl[w * kLd + x] = fma(pht[q], wy, wx) * pc[q];
            Wl[w * kLd + y] = fma(pt[q], wx, wy) * pc[q];
        }
        __syncthreads();
    }
    if (threadIdx.x < kB) {
        if (code) atomicOr(&s_code, code);
        if (nrot) atomicAdd(&s_rot, nrot);
        if (nskip) atomicAdd(&s_skip, nskip);
        if (rank) atomicOr(&a.ctl->rank, 1);
    }
    double *Wg = a.W + (size_t)k * (kB2 * kB2);
    for (int idx = threadIdx.x; idx < kB2 * kB2; idx += 256) {
        const int x = idx / kB2, y = idx % kB2;
        Wg[idx] = Wl[x * kLd + y];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a.C[k] |= s_code;
        a.nrot[k] += (unsigned)s_rot;
        a.nskip[k] += (unsigned)s_skip;
        a.nact[k] += s_rot > 0 ? 1u : 0u;
        a.active[k] = s_rot > 0 ? 1 : 0;
    }
}

// ---------------------------------------------------------------------------
// Update: [G_P | V_P] <- [G_P | V_P] W, 256 rows per workgroup.
// ---------------------------------------------------------------------------
constexpr int kUpdRows = 256;

__global__ __launch_bounds__(256) void block_update_kernel(BlockArgs a)
{
    __shared__ double Wl[kB2 * kLd];
    __shared__ double X[kB2 * kLd];
    __shared__ int cols[kB2];
    const int k = blockIdx.x;
    const int tiles_g = a.ldg / kUpdRows;
    const int t = blockIdx.y;
    if (t == 0 && threadIdx.x == 0 && a.ordering == HSVD_ORD_MODMOD)
        a.S_out[k] = modmod_next(a.S_in[k], a.nb);
    if (!a.active[k]) return;  // no rotation in this pair: W = I
    double *M = t < tiles_g ? a.G : a.V;
    const int row_base = (t < tiles_g ? t : t - tiles_g) * kUpdRows;
    const int2 IJ = outer_pair(a, k);
    if (threadIdx.x < kB2) cols[threadIdx.x] = a.rho[local_pos(threadIdx.x, IJ.x, IJ.y)];
    const double *Wg = a.W + (size_t)k * (kB2 * kB2);
    for (int idx = threadIdx.x; idx < kB2 * kB2; idx += 256) Wl[(idx / kB2) * kLd + idx % kB2] = Wg[idx];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int sub = 0; sub < kUpdRows / 64; ++sub) {
        const int row0 = row_base + sub * 64;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int idx = threadIdx.x + 256 * e;
            const int c = idx >> 6, rr = idx & 63;
            X[c * kLd + rr] = M[(size_t)cols[c] * a.ldg + row0 + rr];
        }
        __syncthreads();
        d4 acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int kk = 0; kk < 16; ++kk) {
            const int xk = kk * 4 + (lane >> 4);
            const double av = X[xk * kLd + wave * 16 + (lane & 15)];
#pragma unroll
            for (int yt = 0; yt < 4; ++yt) {
                const double bv = Wl[xk * kLd + yt * 16 + (lane & 15)];
                acc[yt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[yt], 0, 0, 0);
            }
        }
        __syncthreads();
#pragma unroll
        for (int yt = 0; yt < 4; ++yt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = wave * 16 + (lane >> 4) + 4 * v;
                const int y = yt * 16 + (lane & 15);
                X[y * kLd + row] = acc[yt][v];
            }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int idx = threadIdx.x + 256 * e;
            const int c = idx >> 6, rr = idx & 63;
            M[(size_t)cols[c] * a.ldg + row0 + rr] = X[c * kLd + rr];
        }
        __syncthreads();
    }
}

// Outer stepper start (nb/2 slots, antidiagonal over blocks).
__global__ void block_stepper_init_kernel(int4 *S, int nb)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nb / 2) S[k] = modmod_start(k, nb);
}

// d[pos] = ||G[:, rho[pos]]||^2, one workgroup per position.
__global__ __launch_bounds__(256) void colnorm_pos_kernel(const double *__restrict__ G, int ldg,
                                                          const int *__restrict__ rho,
                                                          double *__restrict__ d)
{
    __shared__ double sh[4];
    const int q = blockIdx.x;
    const double *gc = G + (size_t)rho[q] * ldg;
    double s = 0.0;
    for (int row = threadIdx.x; row < ldg; row += 256) {
        const double x = gc[row];
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

hipError_t launch_block_gram(hipStream_t st, const BlockArgs &a)
{
    block_gram_kernel<<<dim3(a.nb / 2, a.splits), 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_block_inner(hipStream_t st, const BlockArgs &a)
{
    block_inner_kernel<<<a.nb / 2, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_block_update(hipStream_t st, const BlockArgs &a)
{
    const int tiles = (a.ldg / kUpdRows) * (a.V ? 2 : 1);
    block_update_kernel<<<dim3(a.nb / 2, tiles), 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_colnorm_pos(hipStream_t st, const double *G, int ldg, const int *rho, double *d, int r)
{
    colnorm_pos_kernel<<<r, 256, 0, st>>>(G, ldg, rho, d);
    return hipGetLastError();
}

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
