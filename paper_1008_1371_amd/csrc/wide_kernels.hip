// Block path with column blocks of b = 64 (the wide block path), FP64.
//
// The block-oriented method of Sec. 5 with 2b = 128 columns per block pair.
// G and V are kept in position order (column q of the working copies is the
// column at sorted position q; rho maps positions to the input's columns), so
// a block is a contiguous run of 64 columns.  After every sort the columns
// move to their new positions.  One outer step is
//   wide_blk_kernel     the step's block pairs (I, J) from the outer ordering;
//                       the modified modulus stepper advances;
//   Gram                A_P = G_P^T G_P on the FP64 MFMA GEMM (block-pair
//                       form, split over row ranges; gemm_kernels.hip);
//   wide_inner_kernel   the inner rotations of each block pair: A_P in LDS, W
//                       in device memory;
//   update              [G_P | V_P] <- [G_P | V_P] W on the same GEMM, in place.
// The inner ordering is that of the b = 32 path with b = 64: in the first
// outer step of a sweep every pair of the 128 columns once (circle method,
// 127 inner steps), in the others the 64^2 cross pairs
// (x, 64 + ((x + u) mod 64)), 64 inner steps; the full-block method repeats
// circle sweeps until one rotates nothing.
#include "internal.h"

namespace hsvd {

namespace {

constexpr int kWB = kWideB;     // block width
constexpr int kWB2 = 2 * kWB;   // columns of a block pair
constexpr int kWLd = kWB2 + 1;  // LDS row stride of A_P
constexpr int kWT = 1024;       // threads of the inner kernel

}  // namespace

// blk[k] = (I, J) of slot k at outer step `step`; the modified modulus
// stepper's next state into S_out.
__global__ void wide_blk_kernel(int ordering, int nb, int step, const int4 *__restrict__ S_in,
                                int4 *__restrict__ S_out, int2 *__restrict__ blk)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nb / 2) return;
    if (ordering == HSVD_ORD_MODMOD) {
        const int4 s = S_in[k];
        blk[k] = make_int2(s.z, s.w);
        S_out[k] = modmod_next(s, nb);
    } else {
        blk[k] = roundrobin_pair(k, nb, step);
    }
}

// Inner rotations of block pair k.  The partial Grams (column-major 128 x 128,
// both triangles) are summed in split order into A_P in LDS; W, column-major
// (W(x, y) at y * 128 + x), starts as I in device memory.  At an inner step
// every local index belongs to exactly one slot: the first wave evaluates the
// 64 slots' rotations, then thread positions (s1, s2) update the 2 x 2 blocks
// of A_P (rows of slot s1's pair, columns of slot s2's; mirrored blocks in
// mirrored order, so A_P stays exactly symmetric) and the columns of W.
__global__ __launch_bounds__(kWT) void wide_inner_kernel(WideArgs a)
{
    __shared__ double A[kWB2 * kWLd];
    __shared__ double4 prm[kWB];  // (t, c, t or -t, rotated) of each slot
    __shared__ int2 pxy[kWB];     // local indices (x < y) of each slot's pair
    __shared__ int s_any, s_sweep_any;
    const int k = blockIdx.x;
    const int tid = threadIdx.x;
    const int2 IJ = a.blk[k];
    constexpr int kNN = kWB2 * kWB2;
    const double *P = a.partial + (size_t)k * a.splits * kNN;
    for (int idx = tid; idx < kNN; idx += kWT) {
        const int x = idx & (kWB2 - 1), y = idx >> 7;  // element (x, y) at y * 128 + x
        double g = P[idx];
        for (int s = 1; s < a.splits; ++s) g += P[(size_t)s * kNN + idx];
        A[x * kWLd + y] = g;
    }
    double *W = a.W + (size_t)k * kNN;
    for (int idx = tid; idx < kNN; idx += kWT) W[idx] = (idx & (kWB2 - 1)) == (idx >> 7) ? 1.0 : 0.0;
    if (tid == 0) {
        s_any = 0;
        s_sweep_any = 0;
    }
    __syncthreads();

    const bool first = a.first != 0 || a.inner_sweeps > 0;
    const int nsteps = first ? kWB2 - 1 : kWB;
    const int nsweeps = a.inner_sweeps > 0 ? a.inner_sweeps : 1;
    const double tol2 = a.tol * a.tol;
    int code = 0, nrot = 0, nskip = 0, rank = 0;
    double maxt = 0.0;
    unsigned long long tm0 = 0ull, tm1 = 0ull;  // touched local columns 0..63, 64..127
    int mark = 0;
    for (int sw = 0; sw < nsweeps; ++sw) {
        for (int u = 0; u < nsteps; ++u) {
            ++mark;
            if (tid < kWB) {
                const int q = tid;
                const int2 xy = block_inner_pair(q, u, first, kWB);
                const int x = xy.x, y = xy.y;
                const double axx = A[x * kWLd + x], ayy = A[y * kWLd + y], axy = A[x * kWLd + y];
                double t = 0.0, c = 1.0, h = 0.0;
                int rot = 0;
                if (rel_orthogonal_sq(axx, ayy, axy, a.tol, tol2)) {
                    ++nskip;
                } else {
                    const int px = x < kWB ? IJ.x * kWB + x : IJ.y * kWB + x - kWB;
                    const int py = y < kWB ? IJ.x * kWB + y : IJ.y * kWB + y - kWB;
                    const int hyp = ((px < a.p) == (py < a.p)) ? -1 : 1;
                    if (rotation_params_fast(axx, ayy, axy, hyp, t, c)) {
                        rank = 1;
                        t = 0.0;
                        c = 1.0;
                    } else {
                        rot = 1;
                        ++nrot;
                        code |= rotation_code(t, a.tthresh);
                        maxt = fmax(maxt, fabs(t));
                        h = hyp < 0 ? -t : t;
                        if (x < kWB) tm0 |= 1ull << x;
                        else tm1 |= 1ull << (x - kWB);
                        if (y < kWB) tm0 |= 1ull << y;
                        else tm1 |= 1ull << (y - kWB);
                    }
                }
                prm[q] = make_double4(t, c, h, rot ? 1.0 : 0.0);
                pxy[q] = xy;
                if (rot) {
                    s_any = mark;
                    s_sweep_any = sw + 1;
                }
            }
            __syncthreads();
            // no rotation in this inner step: A_P and W unchanged (a late
            // reader of s_any still sees a mismatch: the first wave raises it
            // only after a step with a rotation)
            if (s_any != mark) continue;
#pragma unroll
            for (int qa = 0; qa < (kWB * kWB) / kWT; ++qa) {
                const int pos = tid + kWT * qa;
                const int s1 = pos >> 6, s2 = pos & (kWB - 1);
                const bool cf = s1 <= s2;
                const int2 r1 = pxy[s1], r2 = pxy[s2];
                const double4 pa = prm[cf ? s2 : s1], pq = prm[cf ? s1 : s2];
                const double e00 = A[r1.x * kWLd + r2.x], e01 = A[r1.x * kWLd + r2.y];
                const double e10 = A[r1.y * kWLd + r2.x], e11 = A[r1.y * kWLd + r2.y];
                const double x01 = cf ? e01 : e10, x10 = cf ? e10 : e01;
                const double f00 = fma(pa.z, x01, e00) * pa.y, f01 = fma(pa.x, e00, x01) * pa.y;
                const double f10 = fma(pa.z, e11, x10) * pa.y, f11 = fma(pa.x, x10, e11) * pa.y;
                const double y00 = fma(pq.z, f10, f00) * pq.y, y10 = fma(pq.x, f00, f10) * pq.y;
                const double y01 = fma(pq.z, f11, f01) * pq.y, y11 = fma(pq.x, f01, f11) * pq.y;
                double o01 = cf ? y01 : y10, o10 = cf ? y10 : y01;
                if (s1 == s2 && pa.w != 0.0) {
                    o01 = 0.0;
                    o10 = 0.0;
                }
                A[r1.x * kWLd + r2.x] = y00;
                A[r1.x * kWLd + r2.y] = o01;
                A[r1.y * kWLd + r2.x] = o10;
                A[r1.y * kWLd + r2.y] = y11;
            }
            // W <- W R on the two columns of each slot (rows by consecutive threads)
#pragma unroll
            for (int qw = 0; qw < (kWB * kWB2) / kWT; ++qw) {
                const int item = tid + kWT * qw;
                const int row = item & (kWB2 - 1), wq = item >> 7;
                const double4 pw = prm[wq];
                if (pw.w != 0.0) {
                    const int2 xy = pxy[wq];
                    const double wx = W[xy.x * kWB2 + row], wy = W[xy.y * kWB2 + row];
                    W[xy.x * kWB2 + row] = fma(pw.z, wy, wx) * pw.y;
                    W[xy.y * kWB2 + row] = fma(pw.x, wx, wy) * pw.y;
                }
            }
            __syncthreads();
        }
        if (s_sweep_any < sw + 1) break;
    }
    if (tid < 64) {
        unsigned rot_sum = (unsigned)nrot, skip_sum = (unsigned)nskip;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            code |= __shfl_xor(code, m, 64);
            rank |= __shfl_xor(rank, m, 64);
            rot_sum += __shfl_xor(rot_sum, m, 64);
            skip_sum += __shfl_xor(skip_sum, m, 64);
            maxt = fmax(maxt, __shfl_xor(maxt, m, 64));
            tm0 |= __shfl_xor(tm0, m, 64);
            tm1 |= __shfl_xor(tm1, m, 64);
        }
        if (tid == 0) {
            if (rank) atomicOr(&a.ctl->rank, 1);
            a.maxt[k] = fmax(a.maxt[k], maxt);
            a.C[k] |= code;
            a.nrot[k] += rot_sum;
            a.nskip[k] += skip_sum;
            a.nact[k] += rot_sum > 0 ? 1u : 0u;
            a.ntc[k] += (unsigned)(__popcll(tm0) + __popcll(tm1));
            a.active[k] = rot_sum > 0 ? 1 : 0;
        }
    }
}

// Column moves of the position-ordered working copies: gather (dst column q
// = src column idx[q]) or scatter (dst column idx[q] = src column q), r
// columns of ldg rows; rho_out[q] = rho_in[idx[q]] on a gather when set.
__global__ __launch_bounds__(256) void wide_move_kernel(const double *__restrict__ src, double *__restrict__ dst,
                                                        int ldg, const int *__restrict__ idx, int scatter,
                                                        const int *__restrict__ rho_in, int *__restrict__ rho_out)
{
    const int q = blockIdx.x;
    const int from = scatter ? q : idx[q], to = scatter ? idx[q] : q;
    const double *s = src + (size_t)from * ldg;
    double *d = dst + (size_t)to * ldg;
    for (int row = threadIdx.x; row < ldg; row += 256) d[row] = s[row];
    if (rho_out && threadIdx.x == 0) rho_out[q] = rho_in[idx[q]];
}

__global__ void wide_iota_kernel(int *v, int r)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < r) v[q] = q;
}

hipError_t launch_wide_blk(hipStream_t st, int ordering, int nb, int step, const int4 *S_in, int4 *S_out,
                           int2 *blk)
{
    wide_blk_kernel<<<(nb / 2 + 255) / 256, 256, 0, st>>>(ordering, nb, step, S_in, S_out, blk);
    return hipGetLastError();
}

hipError_t launch_wide_inner(hipStream_t st, const WideArgs &a, int pairs)
{
    wide_inner_kernel<<<pairs, kWT, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_wide_move(hipStream_t st, const double *src, double *dst, int ldg, int r, const int *idx,
                            bool scatter, const int *rho_in, int *rho_out)
{
    wide_move_kernel<<<r, 256, 0, st>>>(src, dst, ldg, idx, scatter ? 1 : 0, rho_in, rho_out);
    return hipGetLastError();
}

hipError_t launch_wide_iota(hipStream_t st, int *v, int r)
{
    wide_iota_kernel<<<(r + 255) / 256, 256, 0, st>>>(v, r);
    return hipGetLastError();
}

}  // namespace hsvd
