// FP64 matrix products of the mixed path's J-re-orthogonalisation on
// 16x16x4 FP64 MFMA.
//
// After the FP32 sweeps the accumulated V is J-orthogonal only to FP32
// accuracy.  The Newton-Schulz iteration that restores it in FP64
// (X <- X (3I - J X^T J X) / 2) and the start of the FP64 refinement
// (G1 = G X) are three products of r x r matrices:
//
//   X^T J X   symmetric; only the upper 128 x 128 tiles are formed and each
//             is written to both triangles (the result is exactly symmetric);
//   X T       and   G X   general products.
//
// One kernel covers them: C = op(A) S B, op(A) = A or A^T, S = I or
// diag(+1 x p, -1 x (K - p)) applied to the rows of B as they are loaded.
// All matrices are column-major FP64.  A workgroup of 256 threads forms a
// 128 x 128 tile of C; each of its four waves a 64 x 64 quarter as 4 x 4
// MFMA tiles of 16 x 16 (64 accumulator registers per lane).  The K
// dimension runs in chunks of 16: the chunk's A and B tiles are staged in
// LDS in the MFMA operand order (element (i, k) of a 16 x 4 operand tile at
// lane i + 16 k), so every operand read is one contiguous 512-byte LDS read,
// and the next chunk's global loads are in flight in registers while the
// current chunk's MFMAs run (two LDS buffers, one barrier per chunk).
//
// The MFMA is issued with the B tile as its first operand, so it computes
// the transpose of the C tile: result lanes then run along the rows of C,
// and each store instruction writes 16 consecutive rows of 4 columns.
//
// Batched use: blockIdx.z is the problem, the operands are offset by fixed
// strides, p may come per problem, and a per-problem flag skips problems
// that take no part in this product.
//
// Block-pair use (the b = 64 block path): the Gram G_P^T G_P of every block
// pair, split over row ranges, and the in-place update G_P <- G_P W address
// the two 64-column blocks of each pair in a position-ordered matrix through
// a column map instead of a problem stride (GemmArgs).
#include "internal.h"

namespace hsvd {

namespace {

typedef double gd2 __attribute__((ext_vector_type(2)));
typedef double gd4 __attribute__((ext_vector_type(4)));

constexpr int kTM = 128;  // rows of a C tile
constexpr int kTN = 128;  // columns of a C tile
constexpr int kTK = 16;   // K chunk
static_assert(kTM == kTN, "square tiles (the symmetric product mirrors them)");

// Position of element (i, k) of a 128 x 16 operand tile in MFMA operand
// order: operand tile (k / 4, i / 16), lane (i % 16) + 16 (k % 4).
__device__ __forceinline__ int frag_pos(int i, int k)
{
    return ((((k >> 2) * (kTM / 16)) + (i >> 4)) << 6) + (i & 15) + ((k & 3) << 4);
}

}  // namespace

template <bool TA, bool SGN, bool SYM>
__global__ __launch_bounds__(256, 2) void gemm_f64_kernel(GemmArgs g)
{
    __shared__ double As[2][kTM * kTK];
    __shared__ double Bs[2][kTN * kTK];
    const int z = blockIdx.z;
    // block-pair form: pair zg, K split ks (see GemmArgs)
    const int zg = g.blk ? z / g.ksplit : z, ks = g.blk ? z % g.ksplit : 0;
    if (g.flag && ((g.flag[zg] != 0) != (g.want != 0))) return;
    const int tiles_m = (g.M + kTM - 1) / kTM, tiles_n = (g.N + kTN - 1) / kTN;
    int tm, tn;
    if (SYM) {
        // upper triangle, tm <= tn, numbered column by column
        const int idx = blockIdx.x;
        int c = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
        while ((c + 1) * (c + 2) / 2 <= idx) ++c;
        while (c * (c + 1) / 2 > idx) --c;
        tn = c;
        tm = idx - c * (c + 1) / 2;
    } else {
        // consecutive workgroups go to different XCDs (round robin over 8):
        // give each XCD a contiguous run of tiles (row-major over C), so the
        // tiles that share a row panel of A share that XCD's L2
        const int tiles = tiles_m * tiles_n;
        int t = blockIdx.x;
        if (tiles % 8 == 0) t = (t % 8) * (tiles / 8) + t / 8;
        tm = t / tiles_n;
        tn = t % tiles_n;
    }
    // A and C may be the same matrix (in-place block-pair update): no
    // restrict on them
    const int mapA = g.map & 1, mapB = g.map & 2, mapC = g.map & 4;
    const size_t koff = (size_t)ks * g.K;  // rows of this K split (transposed A, B)
    const double *A = g.A + (mapA ? (TA ? koff : 0) : (size_t)z * g.sa);
    const double *__restrict__ B = g.B + (mapB ? koff : (size_t)z * g.sb);
    double *C = g.C + (mapC ? 0 : (size_t)z * g.sc);
    const int2 bij = g.blk ? g.blk[zg] : make_int2(0, 0);
    auto mcol = [&](int c) -> size_t {
        return (size_t)(c < g.bw ? bij.x * g.bw + c : bij.y * g.bw + (c - g.bw));
    };
    const int p = g.pvec ? g.pvec[zg] : g.p;
    const int M = g.M, N = g.N, K = g.K;
    const int i0 = tm * kTM, j0 = tn * kTN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    // global loads of one K chunk, 16 bytes per thread and item, 4 items
    gd2 ra[4], rb[4];
    auto gload = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int u = tid + 256 * q;
            if (!TA) {
                // A(i, k) = A[k lda + i]: a wave reads 1 KB of one column
                const int kk = u >> 6, ip = (u & 63) * 2, i = i0 + ip;
                const size_t ca = mapA ? mcol(k0 + kk) : (size_t)(k0 + kk);
                ra[q] = i < M ? *reinterpret_cast<const gd2 *>(A + ca * g.lda + i) : gd2{0.0, 0.0};
            } else {
                // A(i, k) = A[i lda + k]: 8 lanes read 128 bytes of one column
                const int il = u >> 3, kp = (u & 7) * 2, i = i0 + il;
                ra[q] = i < M ? *reinterpret_cast<const gd2 *>(A + (mapA ? mcol(i) : (size_t)i) * g.lda + k0 + kp)
                              : gd2{0.0, 0.0};
            }
            const int jl = u >> 3, kp = (u & 7) * 2, j = j0 + jl;
            gd2 b = j < N ? *reinterpret_cast<const gd2 *>(B + (mapB ? mcol(j) : (size_t)j) * g.ldb + k0 + kp)
                          : gd2{0.0, 0.0};
            if (SGN) {
                if (k0 + kp >= p) b.x = -b.x;
                if (k0 + kp + 1 >= p) b.y = -b.y;
            }
            rb[q] = b;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int u = tid + 256 * q;
            if (!TA) {
                const int kk = u >> 6, ip = (u & 63) * 2;
                *reinterpret_cast<gd2 *>(&As[buf][frag_pos(ip, kk)]) = ra[q];
            } else {
                const int il = u >> 3, kp = (u & 7) * 2;
                As[buf][frag_pos(il, kp)] = ra[q].x;
                As[buf][frag_pos(il, kp + 1)] = ra[q].y;
            }
            const int jl = u >> 3, kp = (u & 7) * 2;
            Bs[buf][frag_pos(jl, kp)] = rb[q].x;
            Bs[buf][frag_pos(jl, kp + 1)] = rb[q].y;
        }
    };

    gd4 acc[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = gd4{0.0, 0.0, 0.0, 0.0};

    const int nk = K / kTK;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kc = 0; kc < nk; ++kc) {
        const int cur = kc & 1;
        if (kc + 1 < nk) gload((kc + 1) * kTK);
#pragma unroll
        for (int kt = 0; kt < kTK / 4; ++kt) {
            double a[4], b[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) a[m] = As[cur][((kt * (kTM / 16) + wm * 4 + m) << 6) + lane];
#pragma unroll
            for (int n = 0; n < 4; ++n) b[n] = Bs[cur][((kt * (kTN / 16) + wn * 4 + n) << 6) + lane];
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < 4; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[n], a[m], acc[m][n], 0, 0, 0);
        }
        if (kc + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }

    // register v of lane l holds C(i0 + 64 wm + 16 m + l % 16, j0 + 64 wn + 16 n + l / 16 + 4 v)
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = i0 + 64 * wm + 16 * m + (lane & 15);
                const int col = j0 + 64 * wn + 16 * n + (lane >> 4) + 4 * v;
                if (row >= M || col >= N) continue;
                const double x = acc[m][n][v];
                if (!SYM) {
                    C[(mapC ? mcol(col) : (size_t)col) * g.ldc + row] = x;
                } else if (row <= col) {
                    // both triangles from the entry with row <= col
                    C[(size_t)col * g.ldc + row] = x;
                    C[(size_t)row * g.ldc + col] = x;
                }
            }
}

hipError_t launch_gemm(hipStream_t st, const GemmArgs &g, int nprob, bool trans_a, bool signed_b, bool symmetric)
{
    if (g.M % 16 || g.N % 16 || g.K % kTK || g.M < 0 || g.N < 0 || g.K < 0 || nprob < 1) return hipErrorInvalidValue;
    if (symmetric && (!trans_a || g.M != g.N || (g.map & 4))) return hipErrorInvalidValue;
    if (g.map && (!g.blk || g.bw < 1 || g.ksplit < 1 || nprob % g.ksplit)) return hipErrorInvalidValue;
    if (g.M == 0 || g.N == 0) return hipSuccess;
    const int tm = (g.M + kTM - 1) / kTM, tn = (g.N + kTN - 1) / kTN;
    const dim3 grid(symmetric ? tm * (tm + 1) / 2 : tm * tn, 1, nprob);
    if (symmetric) {
        if (signed_b) gemm_f64_kernel<true, true, true><<<grid, 256, 0, st>>>(g);
        else gemm_f64_kernel<true, false, true><<<grid, 256, 0, st>>>(g);
    } else if (trans_a) {
        if (signed_b) gemm_f64_kernel<true, true, false><<<grid, 256, 0, st>>>(g);
        else gemm_f64_kernel<true, false, false><<<grid, 256, 0, st>>>(g);
    } else {
        if (signed_b) gemm_f64_kernel<false, true, false><<<grid, 256, 0, st>>>(g);
        else gemm_f64_kernel<false, false, false><<<grid, 256, 0, st>>>(g);
    }
    return hipGetLastError();
}

}  // namespace hsvd
