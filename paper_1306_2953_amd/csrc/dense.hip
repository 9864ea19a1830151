// Orthogonalisation and subspace diagonalisation on gfx950 (Sec. 6).
//
// The N x N matrices are sums over grid points ("block of points"
// contractions, eqs. (7), (9)): S_jk = h^3 sum_p X_pj Y_pk.  They are split
// over chunks of points, each chunk reduced on matrix cores (FP64 MFMA, or
// three BF16 products of the hi/lo split of FP32 data), and the chunk partial
// sums are added in FP64 in a fixed order, so results are bitwise repeatable.
// The rotations psi' = psi X (eqs. (8), (10)) run point-parallel on matrix
// cores, in place.  Cholesky, the triangular inverse and the Jacobi
// eigensolver work on the small FP64 matrices inside one work-group.
#include <cmath>

#include "internal.hpp"
#include "dense.hpp"

namespace rs {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

// bfloat16 with round-to-nearest-even (finite inputs).
__device__ __forceinline__ unsigned short bf16_rne(float x) {
    const uint32_t u = __builtin_bit_cast(uint32_t, x);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) {
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}

// Sum over the 64 lanes of a wave in a fixed butterfly order.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Address of state j at point p in the block layout [j / B][p][j % B].
__device__ __forceinline__ int64_t bidx(int64_t np, int B, int64_t p, int j) {
    return (int64_t)(j / B) * np * B + p * B + (j % B);
}

// ------------------------------------------------------------ Gram FP64
// One work-group per (chunk of points, share of the 16x16 output blocks).
// The chunk is staged KC points at a time in LDS as [point][state]; the
// MFMA A and B fragments of a TN product both read 16 consecutive states of
// one point, so LDS reads are conflict-free.
constexpr int KC64 = 16;
constexpr size_t kJacobiLds = 136 * 1024;   // dynamic LDS for the Jacobi matrix (N <= 130)
constexpr int MAXB = 16;    // 16x16 blocks per wave

template <bool SYRK>
__global__ void __launch_bounds__(256)
gram_f64_kernel(const double *__restrict__ X, const double *__restrict__ Y, int64_t np, int B, int N,
                int N16, int CP, const int2 *__restrict__ blocks, int nblocks, int bps,
                double *__restrict__ partial) {
    extern __shared__ double lds[];
    double *tx = lds;
    double *ty = SYRK ? lds : lds + KC64 * N16;
    const int chunk = blockIdx.x, split = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t p_beg = (int64_t)chunk * CP;
    const int64_t p_end = min<int64_t>(np, p_beg + CP);
    const int b0 = split * bps, b1 = min(nblocks, b0 + bps);
    d4 acc[MAXB];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) acc[i] = d4{0, 0, 0, 0};
    for (int64_t p0 = p_beg; p0 < p_end; p0 += KC64) {
        for (int e = tid; e < KC64 * N16; e += 256) {
            const int p = e / N16, j = e % N16;
            const bool ok = p0 + p < p_end && j < N;
            tx[e] = ok ? X[bidx(np, B, p0 + p, j)] : 0.0;
            if constexpr (!SYRK) ty[e] = ok ? Y[bidx(np, B, p0 + p, j)] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < MAXB; ++i) {
            const int bb = b0 + wave + 4 * i;
            if (bb < b1) {
                const int2 blk = blocks[bb];
#pragma unroll
                for (int kk = 0; kk < KC64 / 4; ++kk) {
                    const int p = kk * 4 + lane / 16;
                    const double a = tx[p * N16 + blk.x * 16 + lane % 16];
                    const double b = ty[p * N16 + blk.y * 16 + lane % 16];
                    acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    double *out = partial + (int64_t)chunk * N16 * N16;
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int bb = b0 + wave + 4 * i;
        if (bb < b1) {
            const int2 blk = blocks[bb];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[(int64_t)(blk.x * 16 + 4 * r + lane / 16) * N16 + blk.y * 16 + lane % 16] = acc[i][r];
        }
    }
}

// ---------------------------------------------------------- Gram BF16x3
// FP32 data split as hi + lo (bfloat16 each); a.b ~ hi.hi + hi.lo + lo.hi
// summed on MFMA 16x16x32 per 32-point stage and accumulated in FP64, plus
// lo.lo: on a diagonal entry
// (a sum of squares) the dropped lo.lo terms are all positive and would bias
// the norms by ~1e-6 relative.  Staged as [state][point] so each lane's 8
// consecutive points (its k-slice) are one 16-byte LDS read.
constexpr int KCB = 32;
constexpr int LDSROW = KCB + 8;   // bf16 elements per state row (padding)

template <bool SYRK>
__global__ void __launch_bounds__(256)
gram_bf16x3_kernel(const float *__restrict__ X, const float *__restrict__ Y, int64_t np, int B, int N,
                   int N16, int CP, const int2 *__restrict__ blocks, int nblocks, int bps,
                   double *__restrict__ partial) {
    extern __shared__ unsigned short ldsh[];
    unsigned short *xh = ldsh, *xl = ldsh + N16 * LDSROW;
    unsigned short *yh = SYRK ? xh : ldsh + 2 * N16 * LDSROW;
    unsigned short *yl = SYRK ? xl : ldsh + 3 * N16 * LDSROW;
    const int chunk = blockIdx.x, split = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t p_beg = (int64_t)chunk * CP;
    const int64_t p_end = min<int64_t>(np, p_beg + CP);
    const int b0 = split * bps, b1 = min(nblocks, b0 + bps);
    d4 acc[MAXB];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) acc[i] = d4{0, 0, 0, 0};
    for (int64_t p0 = p_beg; p0 < p_end; p0 += KCB) {
        for (int e = tid; e < KCB * N16; e += 256) {
            const int p = e / N16, j = e % N16;
            const bool ok = p0 + p < p_end && j < N;
            const float v = ok ? X[bidx(np, B, p0 + p, j)] : 0.0f;
            const unsigned short h = bf16_rne(v);
            xh[j * LDSROW + p] = h;
            xl[j * LDSROW + p] = bf16_rne(v - bf16_to_f(h));
            if constexpr (!SYRK) {
                const float w = ok ? Y[bidx(np, B, p0 + p, j)] : 0.0f;
                const unsigned short g = bf16_rne(w);
                yh[j * LDSROW + p] = g;
                yl[j * LDSROW + p] = bf16_rne(w - bf16_to_f(g));
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < MAXB; ++i) {
            const int bb = b0 + wave + 4 * i;
            if (bb < b1) {
                const int2 blk = blocks[bb];
                const int ka = 8 * (lane / 16);
                const int ra = (blk.x * 16 + lane % 16) * LDSROW + ka;
                const int rb = (blk.y * 16 + lane % 16) * LDSROW + ka;
                const bf8 ah = __builtin_bit_cast(bf8, *(const us8 *)(xh + ra));
                const bf8 al = __builtin_bit_cast(bf8, *(const us8 *)(xl + ra));
                const bf8 bh = __builtin_bit_cast(bf8, *(const us8 *)(yh + rb));
                const bf8 bl = __builtin_bit_cast(bf8, *(const us8 *)(yl + rb));
                // the 32-point products of one stage are summed in FP32 on the
                // matrix core and added to an FP64 accumulator, so rounding of
                // long FP32 sums of same-sign terms cannot bias the result
                f4 t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bl, f4{0, 0, 0, 0}, 0, 0, 0);
                t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, t, 0, 0, 0);
                t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, t, 0, 0, 0);
                t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, t, 0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[i][r] += (double)t[r];
            }
        }
        __syncthreads();
    }
    double *out = partial + (int64_t)chunk * N16 * N16;
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int bb = b0 + wave + 4 * i;
        if (bb < b1) {
            const int2 blk = blocks[bb];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[(int64_t)(blk.x * 16 + 4 * (lane / 16) + r) * N16 + blk.y * 16 + lane % 16] = acc[i][r];
        }
    }
}

// Fixed-order FP64 sum of the chunk partials, one wave per output entry;
// SYRK (mode 1) mirrors the upper blocks, mode 2 symmetrises (M + M^T)/2.
// Output S [N][N] = dv * sum.
__global__ void __launch_bounds__(256)
gram_reduce_kernel(const double *__restrict__ partial, int nchunks, int N, int N16, int mode,
                   double dv, double *__restrict__ S) {
    const int lane = threadIdx.x & 63;
    const int idx = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (idx >= N * N) return;
    const int i = idx / N, j = idx % N;
    auto sum = [&](int a, int b) {
        double s = 0.0;
        for (int c = lane; c < nchunks; c += 64) s += partial[((int64_t)c * N16 + a) * N16 + b];
        return wave_sum(s);
    };
    double v;
    if (mode == 1) {
        const bool up = i / 16 <= j / 16;
        v = sum(up ? i : j, up ? j : i);
    } else if (mode == 2) {
        v = 0.5 * (sum(i, j) + sum(j, i));
    } else {
        v = sum(i, j);
    }
    if (lane == 0) S[idx] = dv * v;
}

// --------------------------------------------------------- rotation FP64
// psi'[p][c] = sum_n psi[p][n] X[n][c], in place.  One wave owns 16 points
// and all N output columns, so every input it needs is read before the
// first store.  MFMA f64 16x16x4: A = psi (16 points x 4 states),
// B = X (4 states x 16 columns), output lane l, reg r -> point 4r + l/16.
constexpr int MAXC64 = 16;   // 16-column blocks per wave (N <= 256)

__global__ void __launch_bounds__(256)
rotate_f64_kernel(double *__restrict__ psi, const double *__restrict__ Xm, int64_t np, int B, int N,
                  int ncb, const int *__restrict__ skip) {
    if (skip && *skip) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t p0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
    if (p0 >= np) return;
    d4 acc[MAXC64];
#pragma unroll
    for (int c = 0; c < MAXC64; ++c) acc[c] = d4{0, 0, 0, 0};
    const int64_t pa = p0 + lane % 16;
    for (int k0 = 0; k0 < N; k0 += 4) {
        const int k = k0 + lane / 16;
        const double a = (pa < np && k < N) ? psi[bidx(np, B, pa, k)] : 0.0;
#pragma unroll
        for (int c = 0; c < MAXC64; ++c) {
            if (c < ncb) {
                const int col = c * 16 + lane % 16;
                const double b = (k < N && col < N) ? Xm[(int64_t)k * N + col] : 0.0;
                acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < MAXC64; ++c) {
        if (c < ncb) {
            const int col = c * 16 + lane % 16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t p = p0 + 4 * r + lane / 16;
                if (p < np && col < N) psi[bidx(np, B, p, col)] = acc[c][r];
            }
        }
    }
}

// ------------------------------------------------------- rotation BF16x3
// FP32 psi and the FP64 matrix X (transposed: xt0/1/2 [c][n]) are both split
// in three bfloat16 terms, a = a0 + a1 + a2, x = x0 + x1 + x2, and the six
// products with a_i x_j, i + j <= 2, are summed on MFMA bf16 16x16x32 in FP32.
// That keeps the rotated field at FP32 accuracy: with only two terms for the
// field, its 2^-17 relative representation error is white noise that the
// kinetic operator amplifies by ~1/h^2 on the next application, and with two
// terms for X every state would be scaled by a common 1 + O(2^-17).
// A = psi (16 points x 32 states, each lane 8 consecutive states of one
// point), B = X (32 states x 16 columns).
__global__ void __launch_bounds__(256)
rotate_bf16x3_kernel(float *__restrict__ psi, const unsigned short *__restrict__ xth,
                     const unsigned short *__restrict__ xtl, const unsigned short *__restrict__ xtm,
                     int64_t np, int B, int N, int N32, int ncb, const int *__restrict__ skip) {
    if (skip && *skip) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t p0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
    if (p0 >= np) return;
    f4 acc[MAXC64];
#pragma unroll
    for (int c = 0; c < MAXC64; ++c) acc[c] = f4{0, 0, 0, 0};
    const int64_t pa = p0 + lane % 16;
    for (int k0 = 0; k0 < N32; k0 += 32) {
        const int kb = k0 + 8 * (lane / 16);
        us8 a0, a1, a2;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const float v = (pa < np && kb + t < N) ? psi[bidx(np, B, pa, kb + t)] : 0.0f;
            const unsigned short h0 = bf16_rne(v);
            const float r1 = v - bf16_to_f(h0);
            const unsigned short h1 = bf16_rne(r1);
            a0[t] = h0;
            a1[t] = h1;
            a2[t] = bf16_rne(r1 - bf16_to_f(h1));
        }
        const bf8 A0 = __builtin_bit_cast(bf8, a0), A1 = __builtin_bit_cast(bf8, a1),
                  A2 = __builtin_bit_cast(bf8, a2);
#pragma unroll
        for (int c = 0; c < MAXC64; ++c) {
            if (c < ncb) {
                const int col = c * 16 + lane % 16;
                const int64_t o = (int64_t)col * N32 + kb;
                const bf8 X0 = __builtin_bit_cast(bf8, *(const us8 *)(xth + o));
                const bf8 X1 = __builtin_bit_cast(bf8, *(const us8 *)(xtm + o));
                const bf8 X2 = __builtin_bit_cast(bf8, *(const us8 *)(xtl + o));
                // smallest terms first
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A2, X0, acc[c], 0, 0, 0);
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, X1, acc[c], 0, 0, 0);
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, X2, acc[c], 0, 0, 0);
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, X0, acc[c], 0, 0, 0);
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, X1, acc[c], 0, 0, 0);
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, X0, acc[c], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < MAXC64; ++c) {
        if (c < ncb) {
            const int col = c * 16 + lane % 16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t p = p0 + 4 * (lane / 16) + r;
                if (p < np && col < N) psi[bidx(np, B, p, col)] = acc[c][r];
            }
        }
    }
}

// X [N][N] (FP64) -> transposed bfloat16 terms x0 + x1 + x2 [N16][N32]
// (each the rounding of what the previous ones leave), zero padded.
__global__ void __launch_bounds__(256)
split_xt_kernel(const double *__restrict__ Xm, int N, int N16, int N32, unsigned short *__restrict__ xth,
                unsigned short *__restrict__ xtl, unsigned short *__restrict__ xtm) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= N16 * N32) return;
    const int c = idx / N32, n = idx % N32;
    const double x = (c < N && n < N) ? Xm[(int64_t)n * N + c] : 0.0;
    const unsigned short h = bf16_rne((float)x);
    const double r1 = x - (double)bf16_to_f(h);
    const unsigned short m = bf16_rne((float)r1);
    const double r2 = r1 - (double)bf16_to_f(m);
    xth[idx] = h;
    xtm[idx] = m;
    xtl[idx] = bf16_rne((float)r2);
}

// ------------------------------------------------------------- Cholesky
// S = U^T U, U upper with positive diagonal (right-looking, one work-group;
// the working copy W lives in LDS when it fits, else in global memory).
// info = 0, or the 1-based column whose pivot is not positive (nothing after
// it is computed).
template <bool LDSW>
__global__ void __launch_bounds__(1024)
cholesky_kernel(const double *__restrict__ S, double *__restrict__ Wg, double *__restrict__ U, int N,
                int *__restrict__ info) {
    extern __shared__ double ldsW[];
    __shared__ double piv;
    __shared__ int bad;
    double *W = LDSW ? ldsW : Wg;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int e = tid; e < N * N; e += nt) {
        W[e] = S[e];
        U[e] = 0.0;
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int k = 0; k < N; ++k) {
        if (tid == 0) {
            const double d = W[k * N + k];
            if (!(d > 0.0) || !isfinite(d)) {
                bad = k + 1;
            } else {
                piv = sqrt(d);
                U[k * N + k] = piv;
                W[k * N + k] = piv;
            }
        }
        __syncthreads();
        if (bad) break;
        const double inv = 1.0 / piv;
        for (int j = k + 1 + tid; j < N; j += nt) {
            const double u = W[k * N + j] * inv;
            W[k * N + j] = u;          // row k of W now holds row k of U
            U[k * N + j] = u;
        }
        __syncthreads();
        // trailing update of the upper triangle: W[i][j] -= U[k][i] U[k][j]
        const int m = N - k - 1;
        for (int e = tid; e < m * m; e += nt) {
            const int i = k + 1 + e / m, j = k + 1 + e % m;
            if (j >= i) W[i * N + j] -= W[k * N + i] * W[k * N + j];
        }
        __syncthreads();
    }
    if (tid == 0) *info = bad;
}

// Inverse of an upper-triangular U: one wave per column j solves U t = e_j
// by back substitution, the inner products split over the 64 lanes and
// summed in a fixed order; the column is kept in LDS.  T = U^-1 is upper
// triangular.  Skipped when info != 0.
__global__ void __launch_bounds__(1024)
trinv_kernel(const double *__restrict__ U, double *__restrict__ T, int N, const int *__restrict__ info) {
    __shared__ double col[16][256];
    if (*info) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    double *t = col[wave];
    for (int j = wave; j < N; j += nw) {
        for (int i = lane; i < N; i += 64) t[i] = 0.0;
        if (lane == 0) t[j] = 1.0 / U[j * N + j];
        __builtin_amdgcn_wave_barrier();
        for (int i = j - 1; i >= 0; --i) {
            double s = 0.0;
            for (int k = i + 1 + lane; k <= j; k += 64) s += U[i * N + k] * t[k];
            s = wave_sum(s);
            if (lane == 0) t[i] = -s / U[i * N + i];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        for (int i = lane; i < N; i += 64) T[i * N + j] = t[i];
        __builtin_amdgcn_wave_barrier();
    }
}

// ------------------------------------------------------ Jacobi eigensolver
// Cyclic parallel Jacobi on a symmetric A (N <= 256, FP64, one work-group).
// Each round rotates N/2 disjoint pairs (round-robin ordering) as
// A <- J^T A J, V <- V J; sweeps repeat until the off-diagonal norm is below
// tol * ||A||_F or max_sweeps is reached.  A lives in LDS when it fits
// (LDSA), else in global memory.  Eigenvalues ascending; each eigenvector's
// largest-magnitude component is made positive.
template <bool LDSA>
__global__ void __launch_bounds__(1024)
jacobi_kernel(double *__restrict__ Ag, double *__restrict__ V, double *__restrict__ evals, int N,
              int max_sweeps, double tol, int *__restrict__ sweeps_out, double *__restrict__ Vt) {
    // A lives in LDS with an odd row stride (column accesses spread over
    // the banks) when it fits, else in place in global memory.  The
    // eigenvector matrix is accumulated transposed (Vt, rows contiguous) so
    // that both passes of a round touch rows only.
    extern __shared__ double ldsA[];
    __shared__ double cs[128], sn[128];
    __shared__ int pp[128], qq[128];
    __shared__ double red[16];
    __shared__ int stop;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    const int ld = LDSA ? N + 1 : N;
    double *A = LDSA ? ldsA : Ag;
    if (LDSA)
        for (int i = wave; i < N; i += nw)
            for (int j = lane; j < N; j += 64) A[i * ld + j] = Ag[i * N + j];
    for (int i = wave; i < N; i += nw)
        for (int j = lane; j < N; j += 64) Vt[i * N + j] = i == j ? 1.0 : 0.0;
    const int M = N + (N & 1);        // even number of players (a dummy when N is odd)
    __syncthreads();
    // Frobenius norms (all entries, then off-diagonal) in a fixed order
    auto block_sum = [&](bool offdiag) {
        double loc = 0.0;
        for (int i = wave; i < N; i += nw)
            for (int j = lane; j < N; j += 64)
                if (!offdiag || i != j) loc += A[i * ld + j] * A[i * ld + j];
        loc = wave_sum(loc);
        if (lane == 0) red[wave] = loc;
        __syncthreads();
        double t = 0.0;
        for (int w2 = 0; w2 < nw; ++w2) t += red[w2];
        __syncthreads();
        return t;
    };
    const double fro = sqrt(block_sum(false));
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        const double off = sqrt(block_sum(true));
        if (tid == 0) stop = !(off > tol * fro);
        __syncthreads();
        if (stop) break;
        for (int r = 0; r < M - 1; ++r) {
            for (int k = tid; k < M / 2; k += blockDim.x) {
                auto pos = [&](int i) { return i == 0 ? 0 : ((i - 1 + r) % (M - 1)) + 1; };
                int p = pos(k), q = pos(M - 1 - k);
                if (p > q) { const int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0;
                if (q < N) {
                    const double apq = A[p * ld + q];
                    if (apq != 0.0) {
                        const double app = A[p * ld + p], aqq = A[q * ld + q];
                        const double th = (aqq - app) / (2.0 * apq);
                        const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        s = t * c;
                    }
                }
                pp[k] = p; qq[k] = q; cs[k] = c; sn[k] = s;
            }
            __syncthreads();
            // columns: A <- A J ; rows of Vt: Vt <- J^T Vt
            for (int k = wave; k < M / 2; k += nw) {
                const int p = pp[k], q = qq[k];
                if (q >= N) continue;
                const double c = cs[k], s = sn[k];
                for (int i = lane; i < N; i += 64) {
                    const double ap = A[i * ld + p], aq = A[i * ld + q];
                    A[i * ld + p] = c * ap - s * aq;
                    A[i * ld + q] = s * ap + c * aq;
                    const double vp = Vt[p * N + i], vq = Vt[q * N + i];
                    Vt[p * N + i] = c * vp - s * vq;
                    Vt[q * N + i] = s * vp + c * vq;
                }
            }
            __syncthreads();
            // rows: A <- J^T A, and the annihilated pivots set exactly to 0
            for (int k = wave; k < M / 2; k += nw) {
                const int p = pp[k], q = qq[k];
                if (q >= N) continue;
                const double c = cs[k], s = sn[k];
                for (int j = lane; j < N; j += 64) {
                    const double ap = A[p * ld + j], aq = A[q * ld + j];
                    A[p * ld + j] = j == q ? 0.0 : c * ap - s * aq;
                    A[q * ld + j] = j == p ? 0.0 : s * ap + c * aq;
                }
            }
            __syncthreads();
        }
    }
    // sort ascending (rank by value, ties by index), normalise signs:
    // one wave per eigenvector
    for (int j = wave; j < N; j += nw) {
        const double d = A[j * ld + j];
        int rank = 0;
        double big = -1.0;
        int arg = 0;
        for (int i = lane; i < N; i += 64) {
            const double e = A[i * ld + i];
            rank += (e < d) || (e == d && i < j);
            const double v = fabs(Vt[j * N + i]);
            if (v > big) { big = v; arg = i; }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            rank += __shfl_xor(rank, o, 64);
            const double ob = __shfl_xor(big, o, 64);
            const int oa = __shfl_xor(arg, o, 64);
            if (ob > big || (ob == big && oa < arg)) { big = ob; arg = oa; }
        }
        if (lane == 0) evals[rank] = d;
        const double sg = Vt[j * N + arg] < 0 ? -1.0 : 1.0;
        for (int i = lane; i < N; i += 64) V[i * N + rank] = sg * Vt[j * N + i];
    }
    if (tid == 0 && sweeps_out) *sweeps_out = sweep;
}

}  // namespace

// ------------------------------------------------------------ launchers
rs_status gram(DenseWork &w, const void *X, const void *Y, int64_t np, int B, int nblk, int dtype,
               int prec, double dv, double *S, int mode, hipStream_t st) {
    const int N = nblk * B;
    const int N16 = (N + 15) / 16 * 16;
    const bool syrk = X == Y;
    const int nb16 = N16 / 16;
    // block list (row block <= col block for the symmetric product)
    std::vector<int2> &bl = syrk ? w.blocks_syrk : w.blocks_full;
    if ((int)bl.size() == 0 || w.blocks_n != N16) {
        w.blocks_syrk.clear();
        w.blocks_full.clear();
        for (int i = 0; i < nb16; ++i)
            for (int j = 0; j < nb16; ++j) {
                w.blocks_full.push_back(int2{i, j});
                if (i <= j) w.blocks_syrk.push_back(int2{i, j});
            }
        w.blocks_n = N16;
        RS_HIP(hipMemcpyAsync(w.d_blocks_syrk.p, w.blocks_syrk.data(), w.blocks_syrk.size() * sizeof(int2),
                              hipMemcpyHostToDevice, st));
        RS_HIP(hipMemcpyAsync(w.d_blocks_full.p, w.blocks_full.data(), w.blocks_full.size() * sizeof(int2),
                              hipMemcpyHostToDevice, st));
    }
    const int nblocks = (int)bl.size();
    const int2 *dbl = syrk ? w.d_blocks_syrk.as<int2>() : w.d_blocks_full.as<int2>();
    const int per_wg = 4 * MAXB;
    const int nsplit = (nblocks + per_wg - 1) / per_wg;
    const int bps = (nblocks + nsplit - 1) / nsplit;
    const bool bf = dtype == RS_F32 && prec == RS_PREC_BF16X3;
    int CP = bf ? 4096 : 2048;
    while ((np + CP - 1) / CP > w.max_chunks) CP *= 2;
    const int nchunks = (int)((np + CP - 1) / CP);
    if ((int64_t)nchunks * N16 * N16 * (int64_t)sizeof(double) > (int64_t)w.partial.bytes)
        return fail(RS_EINVAL, "gram: workspace too small");
    dim3 grid(nchunks, nsplit);
    if (dtype == RS_F64) {
        const size_t lds = (syrk ? 1 : 2) * (size_t)KC64 * N16 * sizeof(double);
        if (syrk)
            hipLaunchKernelGGL(gram_f64_kernel<true>, grid, dim3(256), lds, st, (const double *)X, (const double *)Y,
                               np, B, N, N16, CP, dbl, nblocks, bps, w.partial.as<double>());
        else
            hipLaunchKernelGGL(gram_f64_kernel<false>, grid, dim3(256), lds, st, (const double *)X, (const double *)Y,
                               np, B, N, N16, CP, dbl, nblocks, bps, w.partial.as<double>());
    } else if (bf) {
        const size_t lds = (syrk ? 2 : 4) * (size_t)N16 * LDSROW * sizeof(unsigned short);
        if (syrk)
            hipLaunchKernelGGL(gram_bf16x3_kernel<true>, grid, dim3(256), lds, st, (const float *)X, (const float *)Y,
                               np, B, N, N16, CP, dbl, nblocks, bps, w.partial.as<double>());
        else
            hipLaunchKernelGGL(gram_bf16x3_kernel<false>, grid, dim3(256), lds, st, (const float *)X, (const float *)Y,
                               np, B, N, N16, CP, dbl, nblocks, bps, w.partial.as<double>());
    } else {
        return fail(RS_ENOTSUP, "gram: FP32 data needs RS_PREC_BF16X3");
    }
    RS_HIP(hipGetLastError());
    const int rmode = syrk ? 1 : mode;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3((N * N + 3) / 4), dim3(256), 0, st, w.partial.as<double>(),
                       nchunks, N, N16, rmode, dv, S);
    RS_HIP(hipGetLastError());
    return RS_OK;
}

rs_status rotate(DenseWork &w, void *psi, const double *Xm, int64_t np, int B, int nblk, int dtype, int prec,
                 const int *skip, hipStream_t st) {
    const int N = nblk * B;
    const int N16 = (N + 15) / 16 * 16;
    const int ncb = N16 / 16;
    const unsigned nwg = (unsigned)((np + 63) / 64);
    if (dtype == RS_F64) {
        hipLaunchKernelGGL(rotate_f64_kernel, dim3(nwg), dim3(256), 0, st, (double *)psi, Xm, np, B, N, ncb, skip);
    } else if (prec == RS_PREC_BF16X3) {
        const int N32 = (N + 31) / 32 * 32;
        hipLaunchKernelGGL(split_xt_kernel, dim3((N16 * N32 + 255) / 256), dim3(256), 0, st, Xm, N, N16, N32,
                           w.xth.as<unsigned short>(), w.xtl.as<unsigned short>(), w.xtm.as<unsigned short>());
        RS_HIP(hipGetLastError());
        hipLaunchKernelGGL(rotate_bf16x3_kernel, dim3(nwg), dim3(256), 0, st, (float *)psi,
                           w.xth.as<unsigned short>(), w.xtl.as<unsigned short>(), w.xtm.as<unsigned short>(),
                           np, B, N, N32, ncb, skip);
    } else {
        return fail(RS_ENOTSUP, "rotate: FP32 data needs RS_PREC_BF16X3");
    }
    RS_HIP(hipGetLastError());
    return RS_OK;
}

rs_status cholesky(DenseWork &w, const double *S, double *U, int N, int *info_dev, hipStream_t st) {
    const size_t lds = (size_t)N * N * sizeof(double);
    if (lds <= kJacobiLds) {
        if (!w.chol_lds_set) {
            RS_HIP(hipFuncSetAttribute((const void *)cholesky_kernel<true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kJacobiLds));
            w.chol_lds_set = true;
        }
        hipLaunchKernelGGL(cholesky_kernel<true>, dim3(1), dim3(1024), lds, st, S, w.mwork.as<double>(), U, N,
                           info_dev);
    } else {
        hipLaunchKernelGGL(cholesky_kernel<false>, dim3(1), dim3(1024), 0, st, S, w.mwork.as<double>(), U, N,
                           info_dev);
    }
    RS_HIP(hipGetLastError());
    return RS_OK;
}

rs_status trinv(const double *U, double *T, int N, const int *info_dev, hipStream_t st) {
    hipLaunchKernelGGL(trinv_kernel, dim3(1), dim3(1024), 0, st, U, T, N, info_dev);
    RS_HIP(hipGetLastError());
    return RS_OK;
}

rs_status eigh(DenseWork &w, double *A, double *V, double *evals, int N, hipStream_t st, int max_sweeps) {
    const size_t lds = (size_t)N * (N + 1) * sizeof(double);
    if (lds <= kJacobiLds) {
        if (!w.jacobi_lds_set) {
            RS_HIP(hipFuncSetAttribute((const void *)jacobi_kernel<true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kJacobiLds));
            w.jacobi_lds_set = true;
        }
        hipLaunchKernelGGL(jacobi_kernel<true>, dim3(1), dim3(1024), lds, st, A, V, evals, N, max_sweeps, 1e-15,
                           w.sweeps.as<int>(), w.mwork.as<double>());
    } else {
        hipLaunchKernelGGL(jacobi_kernel<false>, dim3(1), dim3(1024), 0, st, A, V, evals, N, max_sweeps, 1e-15,
                           w.sweeps.as<int>(), w.mwork.as<double>());
    }
    RS_HIP(hipGetLastError());
    return RS_OK;
}

rs_status dense_work_init(DenseWork &w, int64_t np, int max_states) {
    const int N16 = (max_states + 15) / 16 * 16;
    const int N32 = (max_states + 31) / 32 * 32;
    w.max_states = max_states;
    w.max_chunks = 512;
    rs_status s = RS_OK;
    const size_t nb16 = (size_t)(N16 / 16) * (N16 / 16);
    if (!s) s = w.partial.alloc((size_t)w.max_chunks * N16 * N16 * sizeof(double));
    if (!s) s = w.d_blocks_syrk.alloc(nb16 * sizeof(int2));
    if (!s) s = w.d_blocks_full.alloc(nb16 * sizeof(int2));
    if (!s) s = w.mwork.alloc((size_t)max_states * max_states * sizeof(double));
    if (!s) s = w.xth.alloc((size_t)N16 * N32 * sizeof(unsigned short));
    if (!s) s = w.xtl.alloc((size_t)N16 * N32 * sizeof(unsigned short));
    if (!s) s = w.xtm.alloc((size_t)N16 * N32 * sizeof(unsigned short));
    if (!s) s = w.sweeps.alloc(sizeof(int));
    (void)np;
    return s;
}

}  // namespace rs
