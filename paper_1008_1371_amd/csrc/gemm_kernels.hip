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
// One kernel covers them: one workgroup of 256 threads per 128 x 128 tile
// of C, the tile formed by gemm_tile (gemm_device.h, which describes the MFMA
// and LDS scheme).
//
// Batched use: blockIdx.z is the problem, the operands are offset by fixed
// strides, p may come per problem, and a per-problem flag skips problems
// that take no part in this product.
//
// Block-pair use (the b = 64 block path): the Gram G_P^T G_P of every block
// pair, split over row ranges, and the in-place update G_P <- G_P W address
// the two 64-column blocks of each pair in a position-ordered matrix through
// a column map instead of a problem stride (GemmArgs).
#include "gemm_device.h"

namespace hsvd {

using namespace gemm;

template <bool TA, bool SGN, bool SYM>
__global__ __launch_bounds__(256, 2) void gemm_f64_kernel(GemmArgs g)
{
    __shared__ GemmLds L;
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
    gemm_tile<TA, SGN, SYM, false>(g, z, zg, ks, tm, tn, L);
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
