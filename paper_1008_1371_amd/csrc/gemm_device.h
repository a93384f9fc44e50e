// FP64 matrix product tiles on 16x16x4 FP64 MFMA, shared by the grid-wide
// product kernel (gemm_kernels.hip) and the persistent batched solver, which
// forms a small problem's re-orthogonalisation products inside one
// workgroup.  C = op(A) S B, op(A) = A or A^T, S = I or diag(+1 x p, -1 x
// (K - p)) on the rows of B, all column-major FP64.  256 threads form a
// 128 x 128 tile of C; each of their four waves a 64 x 64 quarter as 4 x 4
// MFMA tiles of 16 x 16.  K runs in chunks of 16, staged in LDS in MFMA
// operand order (element (i, k) of a 16 x 4 operand tile at lane i + 16 k,
// so every operand read is one contiguous 512-byte LDS read), the next
// chunk's global loads in flight while the current chunk's MFMAs run (two
// LDS buffers, one barrier per chunk).  The MFMA takes the B tile as its
// first operand, so it computes the transpose of the C tile: result lanes run
// along the rows of C and each store writes 16 consecutive rows of 4 columns.
// A symmetric product (SYM) writes each tile with row <= col to both
// triangles.
#pragma once
#include "internal.h"

namespace hsvd {
namespace gemm {

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

struct GemmLds {
    double As[2][kTM * kTK];
    double Bs[2][kTN * kTK];
};

// Tile (tm, tn) of problem z (zg, ks: block pair and K split of the
// block-pair form, else zg = z, ks = 0).  Every thread of the workgroup calls
// it (barriers); with kGuard only threads 0..255 work.
template <bool TA, bool SGN, bool SYM, bool kGuard>
__device__ __forceinline__ void gemm_tile(const GemmArgs &g, int z, int zg, int ks, int tm, int tn, GemmLds &L)
{
    double(*const As)[kTM * kTK] = L.As;
    double(*const Bs)[kTN * kTK] = L.Bs;
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
    const bool act = !kGuard || tid < 256;  // the tile's 256 threads; others only meet the barriers
    if (act) {
        gload(0);
        sstore(0);
    }
    __syncthreads();
    for (int kc = 0; kc < nk; ++kc) {
        const int cur = kc & 1;
        if (act && kc + 1 < nk) gload((kc + 1) * kTK);
#pragma unroll
        for (int kt = 0; kt < kTK / 4 && act; ++kt) {
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
        if (act && kc + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }
    if (!act) return;

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

}  // namespace gemm
}  // namespace hsvd
