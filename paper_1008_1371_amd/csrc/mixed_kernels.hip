// Helpers of the mixed-precision path: FP32 working copies, and the FP64
// J-re-orthogonalisation of the V accumulated in FP32.
//
// After the FP32 sweeps V32 satisfies V^T J V = J only to FP32 accuracy.  The
// Newton-Schulz iteration for the J-orthogonal factor,
//   X <- X (3I - Y) / 2,  Y = J X^T J X  (the J-adjoint of X times X),
// converges quadratically from X = V32 (promoted) while ||I - Y|| < 1; with X
// J-orthogonal to FP64 accuracy the FP64 refinement sweeps start from
// G1 = G X, V0 = X, so the final V = X V_refine is J-orthogonal in FP64.
// The two products per iteration and G X run on the FP64 MFMA kernels of
// gemm_kernels.hip; these kernels form (3I - J B) / 2 and the residual.
#include "internal.h"

namespace hsvd {

__global__ __launch_bounds__(256) void to_fp32_kernel(const double *__restrict__ G, float *__restrict__ G32,
                                                      float *__restrict__ V32, int ldg, int r)
{
    const int c = blockIdx.x;
    for (int row = threadIdx.x; row < ldg; row += 256) {
        G32[(size_t)c * ldg + row] = (float)G[(size_t)c * ldg + row];
        if (V32) V32[(size_t)c * ldg + row] = row == c ? 1.f : 0.f;
    }
}

__global__ __launch_bounds__(256) void promote_kernel(const float *__restrict__ X32, double *__restrict__ X,
                                                      int ldg, int r)
{
    const int c = blockIdx.x;
    for (int row = threadIdx.x; row < ldg; row += 256) X[(size_t)c * ldg + row] = (double)X32[(size_t)c * ldg + row];
}

// B holds X^T J X (r x r).  Y = J B; B <- (3I - Y) / 2; the largest |Y - I|
// entry is folded into ctl->nsres (non-negative doubles order like their bit
// patterns, so an integer max is exact and order independent).
__global__ __launch_bounds__(256) void ns_form_kernel(double *__restrict__ B, int p, int ldg, int r, Ctl *ctl)
{
    __shared__ double sh[256];
    const int c = blockIdx.x;
    double m = 0.0;
    for (int row = threadIdx.x; row < r; row += 256) {
        const double b = B[(size_t)c * ldg + row];
        const double y = row < p ? b : -b;
        const double id = row == c ? 1.0 : 0.0;
        m = fmax(m, fabs(y - id));
        B[(size_t)c * ldg + row] = (3.0 * id - y) * 0.5;
    }
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        atomicMax(reinterpret_cast<unsigned long long *>(&ctl->nsres),
                  static_cast<unsigned long long>(__double_as_longlong(sh[0])));
}

// dst = src on the r x r block, zero in the padding rows (GEMM results leave
// the rows beyond r unwritten).
__global__ __launch_bounds__(256) void copy_kernel(const double *__restrict__ src, double *__restrict__ dst,
                                                   int ldg, int r)
{
    const int c = blockIdx.x;
    for (int row = threadIdx.x; row < ldg; row += 256)
        dst[(size_t)c * ldg + row] = row < r ? src[(size_t)c * ldg + row] : 0.0;
}

// Column gather Gp[:, k] = G[:, pi[k]] (n x n, leading dimensions ld_in / n).
__global__ __launch_bounds__(256) void gather_cols_kernel(const double *__restrict__ G, int lda,
                                                          const int *__restrict__ pi, double *__restrict__ Gp,
                                                          int n)
{
    const int k = blockIdx.x;
    const double *src = G + (size_t)pi[k] * lda;
    for (int row = threadIdx.x; row < n; row += 256) Gp[(size_t)k * n + row] = src[row];
}

// Outputs of the partitioned solve back to the input column order:
// sigma[pi[k]], lambda[pi[k]], U[:, pi[k]] from column k, V[pi[i], pi[k]] from
// (i, k), perm[q] = pi[perm_p[q]].  grid n
__global__ __launch_bounds__(256) void scatter_outputs_kernel(const int *__restrict__ pi, int n,
                                                              const double *__restrict__ sp,
                                                              const double *__restrict__ Up,
                                                              const double *__restrict__ Vp,
                                                              const double *__restrict__ lp,
                                                              const int *__restrict__ permp,
                                                              double *__restrict__ sigma,
                                                              double *__restrict__ U, int ldu,
                                                              double *__restrict__ V, int ldv,
                                                              double *__restrict__ lambda, int *__restrict__ perm)
{
    const int k = blockIdx.x;
    const int c = pi[k];
    if (threadIdx.x == 0) {
        sigma[c] = sp[k];
        if (lambda) lambda[c] = lp[k];
        if (perm) perm[k] = pi[permp[k]];
    }
    for (int row = threadIdx.x; row < n; row += 256) {
        if (U) U[(size_t)c * ldu + row] = Up[(size_t)k * n + row];
        if (V) V[(size_t)c * ldv + pi[row]] = Vp[(size_t)k * n + row];
    }
}

hipError_t launch_gather_cols(hipStream_t st, const double *G, int lda, const int *pi, double *Gp, int n)
{
    gather_cols_kernel<<<n, 256, 0, st>>>(G, lda, pi, Gp, n);
    return hipGetLastError();
}

hipError_t launch_scatter_outputs(hipStream_t st, const int *pi, int n, const double *sp, const double *Up,
                                  const double *Vp, const double *lp, const int *permp, double *sigma, double *U,
                                  int ldu, double *V, int ldv, double *lambda, int *perm)
{
    scatter_outputs_kernel<<<n, 256, 0, st>>>(pi, n, sp, Up, Vp, lp, permp, sigma, U, ldu, V, ldv, lambda,
                                              perm);
    return hipGetLastError();
}

// Seeded synthetic matrix for the autotuner: uniform in [-1, 1) from the
// splitmix64 hash of (seed, column-major index).
__global__ __launch_bounds__(256) void synth_kernel(double *__restrict__ G, int n, unsigned long long seed)
{
    const int c = blockIdx.x;
    for (int row = threadIdx.x; row < n; row += 256) {
        unsigned long long z = seed + 0x9E3779B97F4A7C15ull * ((unsigned long long)c * n + row + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        G[(size_t)c * n + row] = (double)(z >> 11) * 0x1p-52 - 1.0;
    }
}

hipError_t launch_synth(hipStream_t st, double *G, int n, unsigned long long seed)
{
    synth_kernel<<<n, 256, 0, st>>>(G, n, seed);
    return hipGetLastError();
}

hipError_t launch_to_fp32(hipStream_t st, const double *G, float *G32, float *V32, int ldg, int r)
{
    to_fp32_kernel<<<r, 256, 0, st>>>(G, G32, V32, ldg, r);
    return hipGetLastError();
}

hipError_t launch_promote(hipStream_t st, const float *X32, double *X, int ldg, int r)
{
    promote_kernel<<<r, 256, 0, st>>>(X32, X, ldg, r);
    return hipGetLastError();
}

hipError_t launch_ns_form(hipStream_t st, double *B, int p, int ldg, int r, Ctl *ctl)
{
    ns_form_kernel<<<r, 256, 0, st>>>(B, p, ldg, r, ctl);
    return hipGetLastError();
}

hipError_t launch_copy(hipStream_t st, const double *src, double *dst, int ldg, int r)
{
    copy_kernel<<<r, 256, 0, st>>>(src, dst, ldg, r);
    return hipGetLastError();
}

}  // namespace hsvd
