// Device-side building blocks of the block-column path, shared by the
// per-launch kernels of single and grouped solves (block_kernels.hip) and the
// persistent batched kernel (batch_persist.hip): the MFMA wrappers, the Gram
// of one block pair, the two inner solves of one block pair and the update
// of its columns.  Each takes its block pair index and its LDS explicitly, so
// a caller can run any of them for any pair and share one LDS area between
// them.
#pragma once

#include "internal.h"

namespace hsvd {
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// 16x16x4 MFMA per storage type.  Operand A element (i, k) and operand B
// element (k, j) sit in lane i + 16k resp. j + 16k for both types; the
// accumulator layouts differ (checked on the device):
//   v_mfma_f64_16x16x4f64: register v of lane l holds D(l/16 + 4v, l%16)
//   v_mfma_f32_16x16x4f32: register v of lane l holds D(4(l/16) + v, l%16)
template <typename T>
struct MF;
template <>
struct MF<double> {
    typedef d4 acc;
    static __device__ __forceinline__ acc zero() { return d4{0.0, 0.0, 0.0, 0.0}; }
    static __device__ __forceinline__ acc mma(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct MF<float> {
    typedef f4 acc;
    static __device__ __forceinline__ acc zero() { return f4{0.f, 0.f, 0.f, 0.f}; }
    static __device__ __forceinline__ acc mma(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

constexpr int kB = 32;        // block width b
constexpr int kB2 = 2 * kB;   // columns of a block pair
constexpr int kLd = kB2 + 1;  // LDS row stride (doubles)
constexpr int kMaxSplits = 32; // row splits of the Gram (the host keeps splits <= this)

// Points the argument block at problem blockIdx.z of a batched group; false
// when that problem has already converged.
template <typename T>
__device__ __forceinline__ bool bind_problem(BlockArgsT<T> &a)
{
    if (a.nprob <= 1 && !a.done) return true;
    const int z = blockIdx.z;
    if (a.done && a.done[z]) return false;
    const size_t mat = (size_t)a.ldg * a.r;
    const int pairs = a.nb / 2;
    a.G += z * mat;
    if (a.V) a.V += z * mat;
    a.rho += (size_t)z * a.r;
    a.partial += (size_t)z * pairs * a.splits * (kB2 * kB2);
    a.W += (size_t)z * pairs * (kB2 * kB2);
    a.active += (size_t)z * pairs;
    a.C += (size_t)z * pairs;
    a.nrot += (size_t)z * pairs;
    a.nskip += (size_t)z * pairs;
    a.nact += (size_t)z * pairs;
    a.ntc += (size_t)z * pairs;
    a.maxt += (size_t)z * pairs;
    a.ctl += z;
    if (a.pvec) a.p = a.pvec[z];
    if (a.tolvec) a.tol = a.tolvec[z];
    if (a.tthvec) a.tthresh = a.tthvec[z];
    return true;
}

template <typename T>
__device__ __forceinline__ int2 outer_pair(const BlockArgsT<T> &a, int k)
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
// The Gram matrix is symmetric: only the 10 upper-triangular 16 x 16 tiles
// (xt <= yt) of the 4 x 4 tiling are formed; readers take entry
// (min(x, y), max(x, y)).  An MFMA slice contracts 4 rows; operand A(i, k)
// sits in lane i + 16k, operand B(k, j) in lane j + 16k, so with lane
// (i, k) holding G(row_k, column 16t + i) the same register is the A operand
// of column tile t and the B operand of tile t, and a wave issues all 10
// products from its 4 tile registers.  The rows of a slice need not be
// consecutive: lane (i, k) loads 16 consecutive bytes of column 16t + i
// (V = 16 / sizeof(T) rows) at row offset V k, and element e of that load
// serves slice e.  One load per tile (FP32) or two (FP64, rows + 4V) make a
// chunk of 16 rows; lanes of one load instruction read 64 contiguous bytes
// per column.  No LDS staging: the loads are the MFMA operands.  Wave w
// takes every fourth chunk of the split; the four waves' tiles are summed in
// wave order at the end.
constexpr int kGramTiles = 10;
static __constant__ int kGramTX[kGramTiles] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3};
static __constant__ int kGramTY[kGramTiles] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};

// The Gram of block pair k over the rows of `split`, by the first 256
// threads of the workgroup (waves beyond the fourth only take part in the
// barriers); red: kGramRed elements of LDS.  Every thread must call it.
constexpr int kGramRed = 3 * (kGramTiles / 2) * 256;
template <typename T>
__device__ __forceinline__ void gram_pair(const BlockArgsT<T> &a, int k, int split, T *red)
{
    constexpr int kV = 16 / (int)sizeof(T);  // rows per 16-byte load
    // loads per tile and chunk: FP32 one (16 rows), FP64 two (8 rows each)
    constexpr int NH = sizeof(T) == 4 ? 1 : 2;
    constexpr int kRC = 4 * NH * kV;  // rows per chunk
    typedef T vec __attribute__((ext_vector_type(kV)));
    constexpr int kHalf = kGramTiles / 2;
    const int2 IJ = outer_pair(a, k);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int row_begin = split * a.rows_per_split;
    const int row_end = min(a.ldg, row_begin + a.rows_per_split);
    const int nchunk = (row_end - row_begin) / kRC;
    // byte offsets of this lane's first row in its 4 columns, 32-bit from the
    // uniform base (r, ldg <= 16448: below 2^32 bytes)
    const char *__restrict__ G = reinterpret_cast<const char *>(a.G);
    unsigned off[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
        off[t] = ((unsigned)a.rho[local_pos(16 * t + lr, IJ.x, IJ.y)] * (unsigned)a.ldg +
                  (unsigned)(row_begin + kV * lk)) * (unsigned)sizeof(T);
    typename MF<T>::acc acc[kGramTiles];
#pragma unroll
    for (int q = 0; q < kGramTiles; ++q) acc[q] = MF<T>::zero();
    // no prefetch: the registers go to occupancy instead (measured faster)
    for (int c = wave; c < (wave < 4 ? nchunk : 0); c += 4) {
        vec cur[4][NH];
        const unsigned rb = (unsigned)(c * kRC) * (unsigned)sizeof(T);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int h = 0; h < NH; ++h)
                cur[t][h] = *reinterpret_cast<const vec *>(G + (off[t] + rb + (unsigned)(h * 4 * kV) * sizeof(T)));
#pragma unroll
        for (int h = 0; h < NH; ++h)
#pragma unroll
            for (int e = 0; e < kV; ++e) {
                const T x0 = cur[0][h][e], x1 = cur[1][h][e], x2 = cur[2][h][e], x3 = cur[3][h][e];
                acc[0] = MF<T>::mma(x0, x0, acc[0]);
                acc[1] = MF<T>::mma(x0, x1, acc[1]);
                acc[2] = MF<T>::mma(x0, x2, acc[2]);
                acc[3] = MF<T>::mma(x0, x3, acc[3]);
                acc[4] = MF<T>::mma(x1, x1, acc[4]);
                acc[5] = MF<T>::mma(x1, x2, acc[5]);
                acc[6] = MF<T>::mma(x1, x3, acc[6]);
                acc[7] = MF<T>::mma(x2, x2, acc[7]);
                acc[8] = MF<T>::mma(x2, x3, acc[8]);
                acc[9] = MF<T>::mma(x3, x3, acc[9]);
            }
    }
    // sum over the waves in wave order, five tiles at a time (waves 1..3
    // deposit, wave 0 adds and stores)
    T *out = a.partial + ((size_t)k * a.splits + split) * (kB2 * kB2);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (h) __syncthreads();
        if (wave > 0 && wave < 4) {
#pragma unroll
            for (int j = 0; j < kHalf; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) red[((wave - 1) * kHalf + j) * 256 + v * 64 + lane] = acc[h * kHalf + j][v];
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int j = 0; j < kHalf; ++j) {
                const int q = h * kHalf + j;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    T sum = acc[q][v];
#pragma unroll
                    for (int w = 0; w < 3; ++w) sum += red[(w * kHalf + j) * 256 + v * 64 + lane];
                    const int x = kGramTX[q] * 16 + MF<T>::row(lane, v);
                    const int y = kGramTY[q] * 16 + lr;
                    out[x * kB2 + y] = sum;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Inner solve of one block pair over all pairs of its 2b columns: sweeps of the
// circle method over 2b indices (2b - 1 inner steps of b pairs each).  One
// sweep in the first outer step of a sweep of the block-oriented method;
// repeated until a sweep applies no rotation (at most a.inner_sweeps) in every
// outer step of the full-block method.
//
// A_P and W live in LDS.  At an inner step every local index belongs to
// exactly one slot, so the 2x2 block (s1, s2) of A_P -- rows of slot s1's
// pair, columns of slot s2's -- is read and written by thread (s1, s2) alone,
// and W's columns of slot q by the 32 threads of that slot; the first wave
// evaluates the b rotations.  Mirrored blocks apply row and column operations
// in mirrored order (the transposed block runs the same column-then-row
// sequence), so A_P stays exactly symmetric.  Two barriers per inner step.
// ---------------------------------------------------------------------------
struct CircleLds {
    double A[kB2 * kLd];
    double Wl[kB2 * kLd];
    double4 prm[kB];  // (t, c, t or -t, rotated) of each slot
    int2 pxy[kB];     // local indices (x < y) of each slot's pair
    int s_any, s_sweep_any;
};

// NT threads (a multiple of 64 dividing b^2 = 1024): thread tid takes the A
// blocks and W items at positions tid + NT q, q < 1024 / NT.  Every thread
// must call it (barriers).
template <typename T, int NT>
__device__ __forceinline__ void inner_circle_pair(const BlockArgsT<T> &a, int k, CircleLds &L)
{
    constexpr int KC = (kB * kB) / NT;
    static_assert(KC * NT == kB * kB && NT % 64 == 0, "thread count");
    double *const A = L.A, *const Wl = L.Wl;
    double4 *const prm = L.prm;
    int2 *const pxy = L.pxy;
    int &s_any = L.s_any, &s_sweep_any = L.s_sweep_any;
    const int tid = threadIdx.x;
    const int2 IJ = outer_pair(a, k);

    // A_P = sum of the partial Grams in split order (upper-triangular tiles,
    // vector loads), then every entry (x, y) taken from (min, max)
    {
        typedef T v4 __attribute__((ext_vector_type(4)));
        constexpr int kChunk = sizeof(T) == 4 ? 16 : 8;
#pragma unroll
        for (int qi = 0; qi < KC; ++qi) {
            const int item = tid + NT * qi;
            const int x = item >> 4, y0 = (item & 15) * 4;
            if ((y0 >> 4) >= (x >> 4)) {
                const T *P = a.partial + (size_t)k * a.splits * (kB2 * kB2) + x * kB2 + y0;
                double g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
                for (int base = 0; base < a.splits; base += kChunk) {
                    v4 v[kChunk];
#pragma unroll
                    for (int q = 0; q < kChunk; ++q)
                        v[q] = base + q < a.splits
                                   ? *reinterpret_cast<const v4 *>(P + (size_t)(base + q) * (kB2 * kB2))
                                   : v4{0, 0, 0, 0};
#pragma unroll
                    for (int q = 0; q < kChunk; ++q)
                        if (base + q < a.splits) {
                            const bool first = base + q == 0;
                            g0 = first ? (double)v[q][0] : g0 + (double)v[q][0];
                            g1 = first ? (double)v[q][1] : g1 + (double)v[q][1];
                            g2 = first ? (double)v[q][2] : g2 + (double)v[q][2];
                            g3 = first ? (double)v[q][3] : g3 + (double)v[q][3];
                        }
                }
                double *row = A + x * kLd + y0;
                row[0] = g0;
                row[1] = g1;
                row[2] = g2;
                row[3] = g3;
            }
        }
    }
    if (tid == 0) {
        s_any = 0;
        s_sweep_any = 0;
    }
    __syncthreads();
    for (int idx = tid; idx < kB2 * kB2; idx += NT) {
        const int x = idx >> 6, y = idx & 63;
        if (x > y) A[x * kLd + y] = A[y * kLd + x];
        Wl[x * kLd + y] = x == y ? 1.0 : 0.0;
    }
    __syncthreads();

    int code = 0, nrot = 0, nskip = 0, rank = 0;
    double maxt = 0.0;
    unsigned long long tmask = 0ull;
    const double tol2 = a.tol * a.tol;
    const int nsweeps = a.inner_sweeps > 0 ? a.inner_sweeps : 1;
    int mark = 0;  // index of the current inner step, from 1
    for (int sw = 0; sw < nsweeps; ++sw) {
        for (int u = 0; u < kB2 - 1; ++u) {
            ++mark;
            if (tid < kB) {
                const int q = tid;
                const int2 xy = block_inner_pair(q, u, true, kB);
                const int x = xy.x, y = xy.y;
                const double axx = A[x * kLd + x], ayy = A[y * kLd + y], axy = A[x * kLd + y];
                double t = 0.0, c = 1.0, h = 0.0;
                int rot = 0;
                if (rel_orthogonal_sq(axx, ayy, axy, a.tol, tol2)) {
                    ++nskip;
                } else {
                    const int px_ = local_pos(x, IJ.x, IJ.y), py_ = local_pos(y, IJ.x, IJ.y);
                    const int hyp = ((px_ < a.p) == (py_ < a.p)) ? -1 : 1;
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
                        tmask |= (1ull << x) | (1ull << y);
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
            // no rotation in this inner step: A and W unchanged.  The first wave
            // may already be writing the next step's mark, but only after this
            // step had none, so a late reader still sees a mismatch.
            if (s_any != mark) continue;
#pragma unroll
            for (int qa = 0; qa < KC; ++qa) {
                // A block: rows (x1, y1) by slot s1, columns (x2, y2) by slot s2
                const int pos = tid + NT * qa;
                const int s1 = pos >> 5, s2 = pos & 31;
                const bool cf = s1 <= s2;
                const int2 r1 = pxy[s1], r2 = pxy[s2];
                const double4 pa = prm[cf ? s2 : s1], pq = prm[cf ? s1 : s2];
                const double e00 = A[r1.x * kLd + r2.x], e01 = A[r1.x * kLd + r2.y];
                const double e10 = A[r1.y * kLd + r2.x], e11 = A[r1.y * kLd + r2.y];
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
                A[r1.x * kLd + r2.x] = y00;
                A[r1.x * kLd + r2.y] = o01;
                A[r1.y * kLd + r2.x] = o10;
                A[r1.y * kLd + r2.y] = y11;
            }
#pragma unroll
            for (int qw = 0; qw < KC; ++qw) {
                // W <- W R on the columns of slot wq, rows wr and wr + 32
                const int pos = tid + NT * qw;
                const int wq = pos & 31, wr = pos >> 5;
                const int2 xy = pxy[wq];
                const double4 pw = prm[wq];
                if (pw.w != 0.0) {
#pragma unroll
                    for (int h2 = 0; h2 < 2; ++h2) {
                        const int w = wr + 32 * h2;
                        const double wx = Wl[w * kLd + xy.x], wy = Wl[w * kLd + xy.y];
                        Wl[w * kLd + xy.x] = fma(pw.z, wy, wx) * pw.y;
                        Wl[w * kLd + xy.y] = fma(pw.x, wx, wy) * pw.y;
                    }
                }
            }
            __syncthreads();
        }
        // a sweep without rotations: the block is diagonal.  s_sweep_any only
        // grows (the first wave starts sweep sw + 1, and may raise it, only
        // after sweep sw rotated), so every thread takes the same decision
        // even if it reads the flag late.
        if (s_sweep_any < sw + 1) break;
    }
    T *Wg = a.W + (size_t)k * (kB2 * kB2);
    for (int idx = tid; idx < kB2 * kB2; idx += NT) Wg[idx] = (T)Wl[(idx >> 6) * kLd + (idx & 63)];
    if (tid < 64) {
        // counters of the b slots, reduced within the first wave
        unsigned rot_sum = (unsigned)nrot, skip_sum = (unsigned)nskip;
        unsigned mlo = (unsigned)tmask, mhi = (unsigned)(tmask >> 32);
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            code |= __shfl_xor(code, m, 64);
            rank |= __shfl_xor(rank, m, 64);
            rot_sum += __shfl_xor(rot_sum, m, 64);
            skip_sum += __shfl_xor(skip_sum, m, 64);
            maxt = fmax(maxt, __shfl_xor(maxt, m, 64));
            mlo |= __shfl_xor(mlo, m, 64);
            mhi |= __shfl_xor(mhi, m, 64);
        }
        if (tid == 0) {
            const unsigned long long mask = ((unsigned long long)mhi << 32) | mlo;
            if (rank) atomicOr(&a.ctl->rank, 1);
            a.maxt[k] = fmax(a.maxt[k], maxt);
            a.C[k] |= code;
            a.nrot[k] += rot_sum;
            a.nskip[k] += skip_sum;
            a.nact[k] += rot_sum > 0 ? 1u : 0u;
            a.ntc[k] += (unsigned)__popcll(mask);
            a.active[k] = mask;
        }
    }
}

// Per-slot rotation of the cross kernel in the precision its blocks are held
// in: (t, c) with c negated for an applied trigonometric rotation, decoded to

// (t, |c|, h) with h = -t for such a rotation, h = t otherwise.
template <typename C>
struct SlotRot;
template <>
struct SlotRot<float> {
    typedef float2 packed;
    static __device__ __forceinline__ float2 pack(double t, double c) { return make_float2((float)t, (float)c); }
};
template <>
struct SlotRot<double> {
    typedef double2 packed;
    static __device__ __forceinline__ double2 pack(double t, double c) { return make_double2(t, c); }
};
template <typename C>
struct Rot3 {
    C x, y, z;  // t, |c|, h
};
template <typename C, typename P>
__device__ __forceinline__ Rot3<C> unpack_rot(P r)
{
    return Rot3<C>{r.x, fabs(r.y), r.y < C(0) ? -r.x : r.x};
}

// ---------------------------------------------------------------------------
// Inner solve of one block pair for the cross steps (every outer step but the
// first of a sweep), register-resident.
//
// Slot coordinates: at inner step u slot s pairs local column L_s = s with
// R_s(u) = b + ((s + u) mod b).  The 2x2 block (s1, s2) of A_P has rows
// {L_s1, R_s1(u)} and columns {L_s2, R_s2(u)}; it is held by thread (d, s) =
// (tid / b, tid % b) with s1 = s, s2 = s + d mod b, i.e. by diagonals, so the
// blocks that carry the pivots of the next inner step -- (s, s) and (s, s + 1)
// -- all sit in the first wave.  Since R_s(u + 1) = R_{s+1}(u), moving to the
// next inner step maps block (s1, s2) to
//   LL <- LL,  LR <- LR(s1, s2 + 1),  RL <- RL(s1 + 1, s2),  RR <- RR(s1 + 1, s2 + 1):
// a lane shuffle for RR (same diagonal) and an exchange through LDS for LR and
// RL (neighbouring diagonals), double-buffered so that one barrier per inner
// step suffices.  The first wave (raised priority) evaluates the b rotations
// of the next step from its own registers right after its update and leaves
// them in LDS (double-buffered as well) before that barrier.
//
// Blocks (s1, s2) and (s2, s1) apply their column and row operations in
// mirrored order (columns first iff s1 <= s2), so the two stay exact
// transposes and A stays exactly symmetric.  W, rows {s1, b + s1} by columns
// {L_s2, R_s2(u)}, is held by thread (s1, s2) = (tid / b, tid % b) and shifts
// along s2 by a lane shuffle.
// ---------------------------------------------------------------------------
template <typename T>
struct CrossLds {
    // A_P staging at the start, the two LR / RL exchange buffers in the loop
    double buf[kB2 * kLd];
    // per slot (t, c), c negated for an applied trigonometric rotation (whose
    // h is -t; otherwise h = t): one read per slot and step, the LDS reads
    // being the bulk of an inner step.  The blocks of A_P and W are held in
    // the storage precision T: FP32 in the FP32 sweeps, where the rotations
    // are still computed in FP64 from the FP32 pivots and applied in FP32
    // (W is rounded to T on output in any case).
    typename SlotRot<T>::packed prm[2][kB];
    int rotf[2][kB];  // slot rotated (read by the diagonal blocks)
    int live;         // some cross pair fails the skip test
};

// Every thread must call it (barriers).
template <typename T, int NT>
__device__ __forceinline__ void inner_cross_pair(const BlockArgsT<T> &a, int k, CrossLds<T> &L)
{
    // NT threads; thread tid holds the K blocks (d, s) at positions
    // tid + NT q, q < K: one slot s = tid % b for all of them, diagonals NT/b
    // apart, every slot shift inside the thread's half-wave as with K = 1.
    constexpr int K = (kB * kB) / NT;
    static_assert(K * NT == kB * kB && NT % 64 == 0, "thread count");
    double *const buf = L.buf;
    typename SlotRot<T>::packed(*const prm)[kB] = L.prm;
    int(*const rotf)[kB] = L.rotf;
    int &live = L.live;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int2 IJ = outer_pair(a, k);

    // A_P = sum of the partial Grams in split order.  Work item i sums entries
    // (x, y0 .. y0 + 3), x = i / 16, y0 = 4 (i % 16), of every split with
    // vector loads; only the upper-triangular 16 x 16 tiles hold data.
#pragma unroll
    for (int q = 0; q < K; ++q) {
        typedef T v4 __attribute__((ext_vector_type(4)));
        constexpr int kChunk = sizeof(T) == 4 ? 16 : 8;
        const int item = tid + NT * q;
        const int x = item >> 4, y0 = (item & 15) * 4;
        if ((y0 >> 4) >= (x >> 4)) {
            const T *P = a.partial + (size_t)k * a.splits * (kB2 * kB2) + x * kB2 + y0;
            double g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
            for (int base = 0; base < a.splits; base += kChunk) {
                v4 v[kChunk];
#pragma unroll
                for (int c = 0; c < kChunk; ++c)
                    v[c] = base + c < a.splits
                               ? *reinterpret_cast<const v4 *>(P + (size_t)(base + c) * (kB2 * kB2))
                               : v4{0, 0, 0, 0};
#pragma unroll
                for (int c = 0; c < kChunk; ++c)
                    if (base + c < a.splits) {
                        const bool first = base + c == 0;
                        g0 = first ? (double)v[c][0] : g0 + (double)v[c][0];
                        g1 = first ? (double)v[c][1] : g1 + (double)v[c][1];
                        g2 = first ? (double)v[c][2] : g2 + (double)v[c][2];
                        g3 = first ? (double)v[c][3] : g3 + (double)v[c][3];
                    }
            }
            double *row = buf + x * kLd + y0;
            row[0] = g0;
            row[1] = g1;
            row[2] = g2;
            row[3] = g3;
        }
    }
    if (tid == 0) live = 0;
    __syncthreads();
    const int s = tid & 31;
    const int s1 = s;
    T LL[K], LR[K], RL[K], RR[K];
    T W0L[K], W0R[K], W1L[K], W1R[K];
    int s2[K], lr_cell[K], rl_cell[K];
    bool cf[K];
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const int pos = tid + NT * q;
        const int d = pos >> 5;
        s2[q] = (s + d) & 31;
        cf[q] = s1 <= s2[q];
        // entry (x, y) is read at (min, max) for both mirror positions
        LL[q] = (T)buf[min(s1, s2[q]) * kLd + max(s1, s2[q])];
        LR[q] = (T)buf[s1 * kLd + kB + s2[q]];
        RL[q] = (T)buf[s2[q] * kLd + kB + s1];
        RR[q] = (T)buf[(kB + min(s1, s2[q])) * kLd + kB + max(s1, s2[q])];
        // W block of this position: rows {w1, b + w1} (w1 = d) by columns
        // {L_w2, R_w2} (w2 = s)
        W0L[q] = d == s ? T(1) : T(0);
        W0R[q] = T(0);
        W1L[q] = T(0);
        W1R[q] = d == s ? T(1) : T(0);
        lr_cell[q] = (((d + 1) & 31) << 5) | s;             // position (d + 1, s)
        rl_cell[q] = (((d + 31) & 31) << 5) | ((s + 1) & 31);  // position (d - 1, s + 1)
    }
    const bool diag = tid < kB;  // position (0, s), q = 0
    const double tol2 = a.tol * a.tol;
    {
        // Every cross pair (s, b + s2) of the block pair is the pivot of one
        // inner step.  If none fails the skip test (2.3) on A_P as staged, the
        // first step rotates nothing, A_P stays as it is, and by induction no
        // step rotates: the whole solve is skipped (W = I).  The test takes the
        // entries as the loop holds them (rounded to T).
        int fails = 0;
#pragma unroll
        for (int q = 0; q < K; ++q)
            fails |= rel_orthogonal_sq((T)buf[s * kLd + s], (T)buf[(kB + s2[q]) * kLd + kB + s2[q]], LR[q], a.tol,
                                       tol2)
                         ? 0
                         : 1;
        if (__ballot(fails) != 0ull && lane == 0) atomicOr(&live, 1);
    }
    const int nxt = (lane & 32) | ((lane + 1) & 31);  // lane of (d, s + 1), resp. W column s2 + 1
    T *const xlr = reinterpret_cast<T *>(buf), *const xrl = xlr + 2 * kB * kB;  // [2][b * b] each
    // pivots of slot s (lanes 0 .. b-1 of the first wave, q = 0)
    T pll = LL[0], plr = LR[0], prr = RR[0];
    int code = 0, nrot = 0, nskip = 0, rank = 0;
    double maxt = 0.0;
    unsigned long long tmask = 0ull;  // local columns touched by a rotation (first wave)
    if (tid < 64) __builtin_amdgcn_s_setprio(2);
    __syncthreads();
    const int nsteps = live ? kB : 0;  // the same in every thread
    if (nsteps == 0 && tid < kB) nskip = kB;

    for (int u = 0; u < nsteps; ++u) {
        const int pb = u & 1;
        if (tid < kB) {
            // skip test and rotation evaluated side by side (independent
            // dependency chains), then selected
            const int pl = IJ.x * kB + s, pr = IJ.y * kB + ((s + u) & 31);
            const int hyp = ((pl < a.p) == (pr < a.p)) ? -1 : 1;
            double t, c;
            const int bad = rotation_params_fast(pll, prr, plr, hyp, t, c);
            const bool skip = rel_orthogonal_sq(pll, prr, plr, a.tol, tol2);
            int rot = 0;
            if (skip) {
                ++nskip;
                t = 0.0;
                c = 1.0;
            } else if (bad) {
                rank = 1;
                t = 0.0;
                c = 1.0;
            } else {
                rot = 1;
                ++nrot;
                code |= rotation_code(t, a.tthresh);
                maxt = fmax(maxt, fabs(t));
                tmask |= (1ull << s) | (1ull << (kB + ((s + u) & 31)));
            }
            prm[pb][s] = SlotRot<T>::pack(t, (rot && hyp < 0) ? -c : c);
            rotf[pb][s] = rot;
        }
        __syncthreads();
        // slot s1 = s is common to the thread's positions; W's column slot
        // w2 is s1.  (t, c, h) with h = -t for a trigonometric rotation
        const Rot3<T> p1 = unpack_rot<T>(prm[pb][s1]);
#pragma unroll
        for (int q = 0; q < K; ++q) {
            if (u > 0) {
                // LR and RL of the shift to this step
                LR[q] = xlr[(pb ^ 1) * (kB * kB) + lr_cell[q]];
                RL[q] = xrl[(pb ^ 1) * (kB * kB) + rl_cell[q]];
            }
            const Rot3<T> p2 = unpack_rot<T>(prm[pb][s2[q]]);
            // A block, rows by slot s1, columns by slot s2.  Columns first iff
            // s1 <= s2; otherwise the same column-then-row sequence runs on
            // the transposed block with the slots exchanged, which is the
            // row-then-column order on the block itself.
            const Rot3<T> pa = cf[q] ? p2 : p1, pq = cf[q] ? p1 : p2;
            const T x01 = cf[q] ? LR[q] : RL[q], x10 = cf[q] ? RL[q] : LR[q];
            const T f00 = fma(pa.z, x01, LL[q]) * pa.y, f01 = fma(pa.x, LL[q], x01) * pa.y;
            const T f10 = fma(pa.z, RR[q], x10) * pa.y, f11 = fma(pa.x, x10, RR[q]) * pa.y;
            const T y00 = fma(pq.z, f10, f00) * pq.y, y10 = fma(pq.x, f00, f10) * pq.y;
            const T y01 = fma(pq.z, f11, f01) * pq.y, y11 = fma(pq.x, f01, f11) * pq.y;
            LL[q] = y00;
            RR[q] = y11;
            LR[q] = cf[q] ? y01 : y10;
            RL[q] = cf[q] ? y10 : y01;
        }
        if (diag && rotf[pb][s1]) {
            LR[0] = T(0);
            RL[0] = T(0);
        }
        if (u + 1 < kB) {
#pragma unroll
            for (int q = 0; q < K; ++q) {
                xlr[pb * (kB * kB) + tid + NT * q] = LR[q];
                xrl[pb * (kB * kB) + tid + NT * q] = RL[q];
                RR[q] = __shfl(RR[q], nxt, 64);
            }
            if (tid < 64) {
                // next pivots: a_LL of (s, s), a_LR of (s, s + 1) (lane b + s),
                // a_RR of (s + 1, s + 1) (just shifted in)
                plr = __shfl(LR[0], kB + (lane & 31), 64);
                pll = LL[0];
                prr = RR[0];
            }
        }
        // W <- W R on columns (L_w2, R_w2), then the shift of its R half
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const Rot3<T> pw = p1;
            const T a0 = fma(pw.z, W0R[q], W0L[q]) * pw.y, b0 = fma(pw.x, W0L[q], W0R[q]) * pw.y;
            const T a1 = fma(pw.z, W1R[q], W1L[q]) * pw.y, b1 = fma(pw.x, W1L[q], W1R[q]) * pw.y;
            W0L[q] = a0;
            W1L[q] = a1;
            W0R[q] = __shfl(b0, nxt, 64);
            W1R[q] = __shfl(b1, nxt, 64);
        }
    }
    // after b shifts the slots are back in natural order: R_s = b + s
    T *Wg = a.W + (size_t)k * (kB2 * kB2);
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const int w1 = (tid + NT * q) >> 5, w2 = s;
        Wg[w1 * kB2 + w2] = (T)W0L[q];
        Wg[w1 * kB2 + kB + w2] = (T)W0R[q];
        Wg[(kB + w1) * kB2 + w2] = (T)W1L[q];
        Wg[(kB + w1) * kB2 + kB + w2] = (T)W1R[q];
    }
    if (tid < 64) {
        // counters of the b slots, reduced within the first wave
        unsigned rot_sum = (unsigned)nrot, skip_sum = (unsigned)nskip;
        unsigned mlo = (unsigned)tmask, mhi = (unsigned)(tmask >> 32);
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            code |= __shfl_xor(code, m, 64);
            rank |= __shfl_xor(rank, m, 64);
            rot_sum += __shfl_xor(rot_sum, m, 64);
            skip_sum += __shfl_xor(skip_sum, m, 64);
            maxt = fmax(maxt, __shfl_xor(maxt, m, 64));
            mlo |= __shfl_xor(mlo, m, 64);
            mhi |= __shfl_xor(mhi, m, 64);
        }
        if (tid == 0) {
            const unsigned long long mask = ((unsigned long long)mhi << 32) | mlo;
            if (rank) atomicOr(&a.ctl->rank, 1);
            a.maxt[k] = fmax(a.maxt[k], maxt);
            a.C[k] |= code;
            a.nrot[k] += rot_sum;
            a.nskip[k] += skip_sum;
            a.nact[k] += rot_sum > 0 ? 1u : 0u;
            a.ntc[k] += (unsigned)__popcll(mask);
            a.active[k] = mask;
        }
    }
}


// ---------------------------------------------------------------------------
// Update: [G_P | V_P] <- [G_P | V_P] W.
//
// Computed transposed, (X W)^T = W^T X^T for each 16-row strip X of G_P (or
// V_P): the MFMA B operand (k = column x, j = row) is then 16 consecutive rows
// of one column per 16 lanes, read straight from HBM, and the result lanes
// (i = output column, j = row) store 16 consecutive rows likewise -- no LDS
// staging of the data.  W sits in LDS for all strips of the workgroup.
// ---------------------------------------------------------------------------
// Per storage type: FP32 re-reads W from LDS for every strip and keeps the
// next strip's rows in flight in registers (low register use, high
// occupancy); FP64, at twice the registers per operand, holds all 64 W
// operands in registers across strips instead (measured faster for it).
template <typename T>
struct UpdCfg;
template <>
struct UpdCfg<float> {
    // rows per workgroup: in the solve many pairs update few or no columns,
    // and a launch lasts as long as the workgroups of fully active pairs,
    // whose waves stream their strips one after another; 128 rows (2 strips
    // per wave) measured 29.9 us per launch against 31.7 us at 512 (64 rows:
    // the same as 128)
    static constexpr int rows = 128;
    static constexpr int ld = kB2 + 16;    // LDS row stride of W: a read's 4 row groups in distinct banks
    static constexpr bool w_lds = true;    // W re-read from LDS per strip
    static constexpr int min_blocks = 4;   // workgroups per CU to fit
};
template <>
struct UpdCfg<double> {
    static constexpr int rows = 256;
    static constexpr int ld = kB2 + 1;
    static constexpr bool w_lds = false;
    static constexpr int min_blocks = 1;
};

// Compact update of a block pair whose rotations touched only m <= NC of its
// 2b local columns (list tl, physical columns cols): the other columns of W
// are unit columns and every touched column of W is zero outside the touched
// rows (rotations only combine touched columns), so [G_T | V_T] <- [G_T | V_T]
// W_TT is the whole update.  Same MFMA formulation as the full update with NC
// columns, W_TT zero-padded to NC x NC; only the m touched columns are read
// and written.  NT threads.
template <typename T, int NC, int NT>
__device__ __forceinline__ void update_compact(const BlockArgsT<T> &a, int k, T *__restrict__ M, int row_base,
                                               int nstrips, T *Wl, const int *cols, const int *tl, int m)
{
    constexpr int NW = NT / 64;
    const T *Wg = a.W + (size_t)k * (kB2 * kB2);
    for (int idx = threadIdx.x; idx < NC * NC; idx += NT) {
        const int i = idx / NC, j = idx % NC;
        Wl[idx] = (i < m && j < m) ? Wg[tl[i] * kB2 + tl[j]] : T(0);
    }
    __syncthreads();
    constexpr int KK = NC / 4, YT = NC / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    char *__restrict__ base = reinterpret_cast<char *>(M);
    const unsigned row_off = (unsigned)(row_base + lr) * (unsigned)sizeof(T);
    const unsigned col_bytes = (unsigned)a.ldg * (unsigned)sizeof(T);
#pragma unroll 1
    for (int strip = wave; strip < nstrips; strip += NW) {
        const unsigned rb = (unsigned)(strip * 16) * (unsigned)sizeof(T) + row_off;
        T bv[KK];
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) {
            const int x = 4 * kk + lk;
            bv[kk] = x < m ? *reinterpret_cast<const T *>(base + ((unsigned)cols[x] * col_bytes + rb)) : T(0);
        }
        typename MF<T>::acc acc[YT];
#pragma unroll
        for (int yt = 0; yt < YT; ++yt) acc[yt] = MF<T>::zero();
#pragma unroll
        for (int kk = 0; kk < KK; ++kk)
#pragma unroll
            for (int yt = 0; yt < YT; ++yt)
                acc[yt] = MF<T>::mma(Wl[(4 * kk + lk) * NC + yt * 16 + lr], bv[kk], acc[yt]);
#pragma unroll
        for (int yt = 0; yt < YT; ++yt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int y = yt * 16 + MF<T>::row(lane, v);
                if (y < m) *reinterpret_cast<T *>(base + ((unsigned)cols[y] * col_bytes + rb)) = acc[yt][v];
            }
    }
}

// Rows [row_base, row_base + 16 nstrips) of the 2b columns of block pair k
// in M (G or V) <- themselves times W, by NT threads; mask = the pair's
// touched local columns (nonzero).  kWLds: W re-read from LDS for every
// 16-row strip with the next strip's rows prefetched into registers when
// kPrefetch (else the compiler keeps all 64 W operands in registers across
// strips); kLd: LDS row stride of W.  Every thread must call it (barriers).
template <typename T, int NT, bool kWLds, bool kPrefetch, int kLd>
__device__ __forceinline__ void update_rows(const BlockArgsT<T> &a, int k, T *__restrict__ M, int row_base,
                                            int nstrips, unsigned long long mask, T *Wl, int *cols, int *tl)
{
    constexpr int NW = NT / 64;
    const int2 IJ = outer_pair(a, k);
    const int m = __popcll(mask);
    if (m <= 32) {
        // compact list of the touched local columns, in increasing order
        if (threadIdx.x < kB2 && ((mask >> threadIdx.x) & 1ull)) {
            const int i = __popcll(mask & ((1ull << threadIdx.x) - 1ull));
            tl[i] = threadIdx.x;
            cols[i] = a.rho[local_pos(threadIdx.x, IJ.x, IJ.y)];
        }
        __syncthreads();
        if (m <= 16)
            update_compact<T, 16, NT>(a, k, M, row_base, nstrips, Wl, cols, tl, m);
        else
            update_compact<T, 32, NT>(a, k, M, row_base, nstrips, Wl, cols, tl, m);
        return;
    }
    if (threadIdx.x < kB2) cols[threadIdx.x] = a.rho[local_pos(threadIdx.x, IJ.x, IJ.y)];
    const T *Wg = a.W + (size_t)k * (kB2 * kB2);
    for (int idx = threadIdx.x; idx < kB2 * kB2; idx += NT) Wl[(idx / kB2) * kLd + idx % kB2] = Wg[idx];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    // 32-bit byte offsets from the uniform base (r, ldg <= 16448: below 2^32 bytes).
    // Loads: B(k = x, j = row) = G(row0 + lr, column x = 4kk + lk).
    // Stores: D(i = y, j = row), y = 16yt + MF::row(lane, v).
    char *__restrict__ base = reinterpret_cast<char *>(M);
    const unsigned row_off = (unsigned)(row_base + lr) * (unsigned)sizeof(T);
    const unsigned col_bytes = (unsigned)a.ldg * (unsigned)sizeof(T);
    auto load = [&](int strip, T *bv, const int *cp) {
        const unsigned rb = (unsigned)(strip * 16) * (unsigned)sizeof(T) + row_off;
#pragma unroll
        for (int kk = 0; kk < 16; ++kk)
            bv[kk] = *reinterpret_cast<const T *>(base + ((unsigned)cp[4 * kk + lk] * col_bytes + rb));
    };
    constexpr bool kPre = kWLds && kPrefetch;
    T bv[16], nx[16];
    if (kPre && wave < nstrips) load(wave, bv, cols);
#pragma unroll 1
    for (int strip = wave; strip < nstrips; strip += NW) {
        // With kWLds, the opaque zero wz keeps the compiler from hoisting the
        // column offsets and the 64 W operands into registers across strips.
        int wz = 0;
        if (kWLds) asm volatile("" : "+v"(wz));
        if (kPre)  // next strip in flight during the products; the last re-reads its own rows
            load(strip + NW < nstrips ? strip + NW : strip, nx, cols + wz);
        else
            load(strip, bv, cols + wz);
        const T *Wp = Wl + wz + lk * kLd + lr;
        typename MF<T>::acc acc[4];
#pragma unroll
        for (int yt = 0; yt < 4; ++yt) acc[yt] = MF<T>::zero();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk)
#pragma unroll
            for (int yt = 0; yt < 4; ++yt) {
                // A(i = y, k = x) = W(x, y), x = 4kk + lk, y = 16yt + lr
                const T aw = Wp[4 * kk * kLd + yt * 16];
                acc[yt] = MF<T>::mma(aw, bv[kk], acc[yt]);
            }
        const int *cp = cols + wz;
        const unsigned rb = (unsigned)(strip * 16) * (unsigned)sizeof(T) + row_off;
#pragma unroll
        for (int yt = 0; yt < 4; ++yt)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                *reinterpret_cast<T *>(base + ((unsigned)cp[yt * 16 + MF<T>::row(lane, v)] * col_bytes + rb)) =
                    acc[yt][v];
        if (kPre) {
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) bv[kk] = nx[kk];
        }
    }
}


}  // namespace hsvd
