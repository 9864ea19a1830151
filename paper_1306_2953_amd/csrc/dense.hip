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
#include <algorithm>
#include <cmath>

#include "dense.hpp"
#include "internal.hpp"

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
constexpr int kMaxSweeps = 30;             // Jacobi sweep cap (rotation record size)
constexpr int MAXB = 16;    // 16x16 blocks per wave

// NBW > 0: every wave owns exactly NBW blocks (b1 - b0 == 4 * NBW), and the
// MFMAs run k outer, blocks inner, so consecutive ones feed independent
// accumulators; NBW == 0: any share, one block's k steps at a time.
template <bool SYRK, int NBW>
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
    constexpr int NB = NBW > 0 ? NBW : 1;
    int bx[NB], by[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int2 blk = NBW > 0 ? blocks[b0 + wave + 4 * i] : int2{0, 0};
        bx[i] = blk.x;
        by[i] = blk.y;
    }
    for (int64_t p0 = p_beg; p0 < p_end; p0 += KC64) {
        for (int e = tid; e < KC64 * N16; e += 256) {
            const int p = e / N16, j = e % N16;
            const bool ok = p0 + p < p_end && j < N;
            tx[e] = ok ? X[bidx(np, B, p0 + p, j)] : 0.0;
            if constexpr (!SYRK) ty[e] = ok ? Y[bidx(np, B, p0 + p, j)] : 0.0;
        }
        __syncthreads();
        if constexpr (NBW > 0) {
#pragma unroll
            for (int kk = 0; kk < KC64 / 4; ++kk) {
                const int p = kk * 4 + lane / 16;
#pragma unroll
                for (int i = 0; i < NBW; ++i) {
                    const double a = tx[p * N16 + bx[i] * 16 + lane % 16];
                    const double b = ty[p * N16 + by[i] * 16 + lane % 16];
                    acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
                }
            }
        } else {
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

// ------------------------------------------ Gram FP64, 4 blocks of 32 states
// Register-fed form for N = 128 in blocks of B = 32 (the eigensolver's
// shape).  A lane reads 16 bytes of a point row: states 2m and 2m + 1 of one
// block (m = lane % 16) at point 4t + lane / 16 of k-step t, so a wave's
// load covers 4 whole rows.  The even and the odd states of block b act as
// two 16-state tiles, 2b and 2b + 1: one load feeds both MFMA fragments, and
// no LDS stage or barrier is needed.  Loads run kGramDepth k-steps ahead of
// the MFMAs that use them.  Reads past the chunk's end come back as zeros
// (buffer bounds), so every chunk runs whole groups of k-steps.
//  - symmetric (X == Y): two waves per chunk; each reads all four blocks
//    and owns 18 of the 36 tile pairs t1 <= t2 (lists 0 and 1);
//  - general: four waves per chunk; wave w reads X blocks 2(w/2), 2(w/2)+1
//    and Y blocks 2(w%2), 2(w%2)+1 and owns their 16 tile pairs (list 2,
//    fragments 0-3 from X, 4-7 from Y).
// A fragment index f names register half f % 2 of the load from block slot
// f / 2.  The partial of tile pair (t1, t2) holds entry (i, j), i in tile t1.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
__device__ __forceinline__ rsrc_t make_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
constexpr int kGramDepth = 4;
constexpr int kGramPairs[3][18][2] = {
    {{0, 0}, {0, 1}, {1, 1}, {2, 2}, {2, 3}, {3, 3}, {0, 2}, {0, 3}, {1, 2},
     {1, 3}, {4, 6}, {4, 7}, {5, 6}, {5, 7}, {0, 4}, {0, 5}, {1, 4}, {1, 5}},
    {{4, 4}, {4, 5}, {5, 5}, {6, 6}, {6, 7}, {7, 7}, {0, 6}, {0, 7}, {1, 6},
     {1, 7}, {2, 4}, {2, 5}, {3, 4}, {3, 5}, {2, 6}, {2, 7}, {3, 6}, {3, 7}},
    {{0, 4}, {0, 5}, {0, 6}, {0, 7}, {1, 4}, {1, 5}, {1, 6}, {1, 7},
     {2, 4}, {2, 5}, {2, 6}, {2, 7}, {3, 4}, {3, 5}, {3, 6}, {3, 7}, {0, 0}, {0, 0}}};

typedef double d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void gram_r32_load(const rsrc_t (&rs)[4], uint32_t lane_off, int t, d2 (&b)[4]) {
    const int off = (int)(lane_off + (uint32_t)t * 1024u);
#pragma unroll
    for (int f = 0; f < 4; ++f)
        b[f] = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(rs[f], off, 0, 0));
}
// The first kGramDepth k-steps' loads are issued by the caller (before any
// branch on the wave's list, so that they stay in k-step order).  The
// scheduler barriers keep the loads in that order, so the wait before a
// step's MFMAs leaves the later steps' loads in flight.
template <int L, int NP>
__device__ __forceinline__ void gram_r32_wave(const rsrc_t (&rs)[4], int nk, uint32_t lane_off,
                                              d2 (&buf)[kGramDepth][4], const int (&tile)[8],
                                              double *__restrict__ out) {
    d4 acc[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) acc[i] = d4{0, 0, 0, 0};
    for (int t0 = 0; t0 < nk; t0 += kGramDepth) {
#pragma unroll
        for (int j = 0; j < kGramDepth; ++j) {
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const int f1 = kGramPairs[L][i][0], f2 = kGramPairs[L][i][1];
                acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(buf[j][f1 >> 1][f1 & 1], buf[j][f2 >> 1][f2 & 1],
                                                              acc[i], 0, 0, 0);
            }
            gram_r32_load(rs, lane_off, t0 + j + kGramDepth, buf[j]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    const int g = (int)(threadIdx.x & 63) >> 4, m = threadIdx.x & 15;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const int t1 = tile[kGramPairs[L][i][0]], t2 = tile[kGramPairs[L][i][1]];
        const int col = (t2 >> 1) * 32 + 2 * m + (t2 & 1);
#pragma unroll
        for (int r = 0; r < 4; ++r)
            out[((t1 >> 1) * 32 + 2 * (4 * r + g) + (t1 & 1)) * 128 + col] = acc[i][r];
    }
}

template <bool SYRK>
__global__ void __launch_bounds__(SYRK ? 128 : 256) __attribute__((amdgpu_waves_per_eu(2)))
gram_f64_r32_kernel(const double *__restrict__ X, const double *__restrict__ Y, int64_t np, int64_t CP,
                    double *__restrict__ partial) {
    const int chunk = blockIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int64_t p_beg = (int64_t)chunk * CP;
    const int64_t npts = min<int64_t>(np, p_beg + CP) - p_beg;
    const uint32_t bytes = (uint32_t)(npts * 256);
    const int nk = (int)((npts + 4 * kGramDepth - 1) / (4 * kGramDepth)) * kGramDepth;
    const uint32_t lane_off = (uint32_t)((lane >> 4) * 256 + (lane & 15) * 16);
    double *out = partial + (int64_t)chunk * 128 * 128;
    rsrc_t rs[4];
    int tile[8];
    if constexpr (SYRK) {
#pragma unroll
        for (int f = 0; f < 4; ++f) rs[f] = make_rsrc(X + (f * np + p_beg) * 32, bytes);
#pragma unroll
        for (int f = 0; f < 8; ++f) tile[f] = f;
    } else {
        const int xa = 2 * (wave >> 1), yb = 2 * (wave & 1);
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            rs[f] = make_rsrc(X + ((xa + f) * np + p_beg) * 32, bytes);
            rs[2 + f] = make_rsrc(Y + ((yb + f) * np + p_beg) * 32, bytes);
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            tile[f] = 2 * xa + f;
            tile[4 + f] = 2 * yb + f;
        }
    }
    d2 buf[kGramDepth][4];
#pragma unroll
    for (int j = 0; j < kGramDepth; ++j) {
        gram_r32_load(rs, lane_off, j, buf[j]);
        __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (SYRK) {
        if (wave == 0) gram_r32_wave<0, 18>(rs, nk, lane_off, buf, tile, out);
        else gram_r32_wave<1, 18>(rs, nk, lane_off, buf, tile, out);
    } else {
        gram_r32_wave<2, 16>(rs, nk, lane_off, buf, tile, out);
    }
}

// ------------------------------------ Gram BF16x3, 4 blocks of 32 states
// The FP32 form of the register-fed product above (the same even / odd
// state tiles).  MFMA bf16 16x16x32 takes 8 k-values per lane: lane (g, m),
// g = lane / 16, reads states 2m and 2m + 1 of a block (8 bytes) at points
// 32t + 8g + s, s = 0..7, of k-step t, and splits each value x into bf16
// hi = rn(x) and lo = rn(x - hi) in registers.  A tile pair's four products
// hi.hi, hi.lo, lo.hi and lo.lo of one k-step are summed in FP32 on the
// matrix core and added to an FP64 accumulator, so the running sums carry
// no FP32 rounding.  With FP64 accumulators a wave holds 9 tile pairs:
//  - symmetric: four waves per chunk, lists 0-3 (each within three blocks;
//    the loads of a block a list does not use are dropped by the compiler);
//  - general: eight waves per chunk; wave w reads X block w / 2 (fragments
//    0, 1) and Y blocks 2(w%2), 2(w%2)+1 (fragments 4-7): 8 tile pairs.
// The next k-step's loads are in flight while the current one is split and
// multiplied.
constexpr int kGramBfPairs[5][9][2] = {
    {{0, 0}, {0, 1}, {1, 1}, {2, 2}, {2, 3}, {3, 3}, {4, 4}, {4, 5}, {5, 5}},
    {{6, 6}, {6, 7}, {7, 7}, {0, 6}, {0, 7}, {1, 6}, {1, 7}, {2, 6}, {2, 7}},
    {{0, 2}, {0, 3}, {1, 2}, {1, 3}, {0, 4}, {0, 5}, {1, 4}, {1, 5}, {2, 4}},
    {{2, 5}, {3, 4}, {3, 5}, {4, 6}, {4, 7}, {5, 6}, {5, 7}, {3, 6}, {3, 7}},
    {{0, 4}, {0, 5}, {0, 6}, {0, 7}, {1, 4}, {1, 5}, {1, 6}, {1, 7}, {0, 0}}};

template <int L, int NP>
__device__ __forceinline__ void gram_bf_r32_wave(const rsrc_t (&rs)[4], int nk, uint32_t lane_off,
                                                 const int (&tile)[8], double *__restrict__ out) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    f2 raw[4][8];
    d4 acc[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) acc[i] = d4{0, 0, 0, 0};
    auto load = [&](int t) {
        const uint32_t off = lane_off + (uint32_t)t * 4096u;
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int k = 0; k < 8; ++k)
                raw[f][k] = __builtin_bit_cast(
                    f2, __builtin_amdgcn_raw_buffer_load_b64(rs[f], (int)(off + (uint32_t)k * 128u), 0, 0));
    };
    load(0);
    for (int t = 0; t < nk; ++t) {
        bf8 hi[8], lo[8];
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int k = 0; k < 8; ++k)
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const float x = raw[f][k][e];
                    const __bf16 h = (__bf16)x;
                    hi[2 * f + e][k] = h;
                    lo[2 * f + e][k] = (__bf16)(x - (float)h);
                }
        load(t + 1);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int f1 = kGramBfPairs[L][i][0], f2 = kGramBfPairs[L][i][1];
            f4 p = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lo[f1], lo[f2], f4{0, 0, 0, 0}, 0, 0, 0);
            p = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi[f1], lo[f2], p, 0, 0, 0);
            p = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lo[f1], hi[f2], p, 0, 0, 0);
            p = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi[f1], hi[f2], p, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][r] += (double)p[r];
        }
    }
    const int g = (int)(threadIdx.x & 63) >> 4, m = threadIdx.x & 15;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const int t1 = tile[kGramBfPairs[L][i][0]], t2 = tile[kGramBfPairs[L][i][1]];
        const int col = (t2 >> 1) * 32 + 2 * m + (t2 & 1);
#pragma unroll
        for (int r = 0; r < 4; ++r)
            out[((t1 >> 1) * 32 + 2 * (4 * g + r) + (t1 & 1)) * 128 + col] = acc[i][r];
    }
}

template <bool SYRK>
__global__ void __launch_bounds__(SYRK ? 256 : 512) __attribute__((amdgpu_waves_per_eu(2)))
gram_bf_r32_kernel(const float *__restrict__ X, const float *__restrict__ Y, int64_t np, int64_t CP,
                   double *__restrict__ partial) {
    const int chunk = blockIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int64_t p_beg = (int64_t)chunk * CP;
    const int64_t npts = min<int64_t>(np, p_beg + CP) - p_beg;
    const uint32_t bytes = (uint32_t)(npts * 128);
    const int nk = (int)((npts + 31) / 32);
    const uint32_t lane_off = (uint32_t)((lane >> 4) * 8 * 128 + (lane & 15) * 8);
    double *out = partial + (int64_t)chunk * 128 * 128;
    rsrc_t rs[4];
    int tile[8];
    if constexpr (SYRK) {
#pragma unroll
        for (int f = 0; f < 4; ++f) rs[f] = make_rsrc(X + (f * np + p_beg) * 32, bytes);
#pragma unroll
        for (int f = 0; f < 8; ++f) tile[f] = f;
        if (wave == 0) gram_bf_r32_wave<0, 9>(rs, nk, lane_off, tile, out);
        else if (wave == 1) gram_bf_r32_wave<1, 9>(rs, nk, lane_off, tile, out);
        else if (wave == 2) gram_bf_r32_wave<2, 9>(rs, nk, lane_off, tile, out);
        else gram_bf_r32_wave<3, 9>(rs, nk, lane_off, tile, out);
    } else {
        const int xa = wave >> 1, yb = 2 * (wave & 1);
        rs[0] = rs[1] = make_rsrc(X + (xa * np + p_beg) * 32, bytes);
        rs[2] = make_rsrc(Y + (yb * np + p_beg) * 32, bytes);
        rs[3] = make_rsrc(Y + ((yb + 1) * np + p_beg) * 32, bytes);
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            tile[f] = 2 * xa + (f & 1);
            tile[4 + f] = 2 * yb + f;
        }
        gram_bf_r32_wave<4, 8>(rs, nk, lane_off, tile, out);
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

// VEC (B a multiple of 4): a thread stages 4 consecutive points x 4
// consecutive states, read as four 16-byte loads (8 threads cover 128
// contiguous bytes of a point row) and written as one 8-byte LDS store per
// state and term (4 points of one state row).
template <bool SYRK, bool VEC>
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
    // split v into hi + lo bfloat16 for 4 points of one state, packed
    auto put4 = [&](const f4 (&v)[4], int s, unsigned short *hi, unsigned short *lo, int off) {
        unsigned short h[4], l[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            h[t] = bf16_rne(v[t][s]);
            l[t] = bf16_rne(v[t][s] - bf16_to_f(h[t]));
        }
        typedef unsigned int u2 __attribute__((ext_vector_type(2)));
        *(u2 *)(hi + off) = u2{(unsigned)h[0] | ((unsigned)h[1] << 16), (unsigned)h[2] | ((unsigned)h[3] << 16)};
        *(u2 *)(lo + off) = u2{(unsigned)l[0] | ((unsigned)l[1] << 16), (unsigned)l[2] | ((unsigned)l[3] << 16)};
    };
    for (int64_t p0 = p_beg; p0 < p_end; p0 += KCB) {
        if constexpr (VEC) {
            for (int q = tid; q < 2 * N16; q += 256) {
                const int pq = q & 7, j0 = 4 * (q >> 3);
                f4 v[4], w[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int64_t p = p0 + 4 * pq + t;
                    const bool ok = p < p_end && j0 < N;
                    v[t] = ok ? *(const f4 *)(X + bidx(np, B, p, j0)) : f4{0, 0, 0, 0};
                    if constexpr (!SYRK) w[t] = ok ? *(const f4 *)(Y + bidx(np, B, p, j0)) : f4{0, 0, 0, 0};
                }
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int off = (j0 + s) * LDSROW + 4 * pq;
                    put4(v, s, xh, xl, off);
                    if constexpr (!SYRK) put4(w, s, yh, yl, off);
                }
            }
        } else {
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

// Two-pass fixed-order FP64 sum of the chunk partials.  Pass 1: thread
// (entry e of the N16 x N16 partial, group g) sums chunks g*cpg .. in order
// (consecutive threads read consecutive entries of one chunk); pass 2: one
// thread per output entry sums the groups in order, mirrors (SYRK, mode 1)
// or symmetrises (mode 2), and scales by dv.
constexpr int kRedGroups = kGramRedGroups;
__global__ void __launch_bounds__(256)
gram_reduce1_kernel(const double *__restrict__ partial, int nchunks, int cpg, int64_t ne,
                    double *__restrict__ red) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int g = blockIdx.y;
    if (e >= ne) return;
    const int c0 = g * cpg, c1 = min(nchunks, c0 + cpg);
    double sum = 0.0;
    for (int c = c0; c < c1; ++c) sum += partial[(int64_t)c * ne + e];
    red[(int64_t)g * ne + e] = sum;
}
__global__ void __launch_bounds__(256)
gram_reduce2_kernel(const double *__restrict__ red, int ng, int N, int N16, int mode, double dv,
                    double *__restrict__ S) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= N * N) return;
    const int i = idx / N, j = idx % N;
    const int64_t ne = (int64_t)N16 * N16;
    auto sum = [&](int a, int b) {
        double v = 0.0;
        for (int g = 0; g < ng; ++g) v += red[g * ne + (int64_t)a * N16 + b];
        return v;
    };
    double v;
    if (mode == 1) {
        const bool up = i / 16 <= j / 16;
        v = sum(up ? i : j, up ? j : i);
    } else if (mode == 3) {     // tiles of the even / odd states of 32-state blocks
        const bool up = 2 * (i / 32) + (i & 1) <= 2 * (j / 32) + (j & 1);
        v = sum(up ? i : j, up ? j : i);
    } else if (mode == 2) {
        v = 0.5 * (sum(i, j) + sum(j, i));
    } else {
        v = sum(i, j);
    }
    S[idx] = dv * v;
}

// --------------------------------------------------------- rotation FP64
// psi'[p][c] = sum_n psi[p][n] X[n][c], in place.  MFMA f64 16x16x4:
// A = psi (16 points x 4 states), B = X (4 states x 16 columns), output
// lane l, reg r -> point 4r + l/16.
constexpr int MAXC64 = 16;   // 16-column blocks (N <= 256)
// A work-group of 8 waves owns 8 * 16 * MT points and all N <= 16 * MAXC
// output columns, so every input it needs is read before the first store.
// Rows of X arrive through LDS in chunks of KR rows shared by the 8 waves
// (X is read once per work-group); MT point tiles per wave reuse each B
// operand.
constexpr int KR = 32;
template <int MT, int MAXC>
__global__ void __launch_bounds__(512)
rotate_f64_lds_kernel(double *__restrict__ psi, const double *__restrict__ Xm, int64_t np, int B, int N,
                      int ncb, const int *__restrict__ skip) {
    extern __shared__ double xs[];              // [KR][ncb * 16 + 4]
    if (skip && *skip) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ld = ncb * 16 + 4;
    const int64_t pw = ((int64_t)blockIdx.x * 8 + wave) * 16 * MT;
    d4 acc[MT][MAXC];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int c = 0; c < MAXC; ++c) acc[m][c] = d4{0, 0, 0, 0};
    for (int kc = 0; kc < N; kc += KR) {
        __syncthreads();
        for (int e = threadIdx.x; e < KR * ncb * 16; e += 512) {
            const int r = e / (ncb * 16), col = e % (ncb * 16), k = kc + r;
            xs[r * ld + col] = (k < N && col < N) ? Xm[(int64_t)k * N + col] : 0.0;
        }
        __syncthreads();
#pragma unroll 2
        for (int k4 = 0; k4 < KR; k4 += 4) {
            const int k = kc + k4 + lane / 16;
            double a[MT];
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                const int64_t pa = pw + m * 16 + lane % 16;
                a[m] = (pa < np && k < N) ? psi[bidx(np, B, pa, k)] : 0.0;
            }
#pragma unroll
            for (int c = 0; c < MAXC; ++c) {
                if (c < ncb) {
                    const double b = xs[(k4 + lane / 16) * ld + c * 16 + lane % 16];
#pragma unroll
                    for (int m = 0; m < MT; ++m)
                        acc[m][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b, acc[m][c], 0, 0, 0);
                }
            }
        }
    }
    // every read of this work-group's points is done before the first store
    __syncthreads();
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int c = 0; c < MAXC; ++c) {
            if (c < ncb) {
                const int col = c * 16 + lane % 16;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t p = pw + m * 16 + 4 * r + lane / 16;
                    if (p < np && col < N) psi[bidx(np, B, p, col)] = acc[m][c][r];
                }
            }
        }
}

// The same rotation with row-contiguous loads of psi (B a multiple of 16):
// in each block of 16 states, lane group j = lane / 16 of a wave holds
// states 4j .. 4j+3 of its point (one 32-byte load), so a wave reads 16
// points x 128 contiguous bytes; MFMA step i of the block takes state
// 4j + i from every group and the X rows in the same order, which sums the
// same 16 products.  Two register buffers alternate so that the next
// block's loads are in flight while the current one is multiplied.
constexpr int kRotMT = 2;    // 16-point row blocks per wave in the persistent rotation
template <int MT, int MAXC>
__global__ void __launch_bounds__(512)
rotate_f64_vec_kernel(double *__restrict__ psi, const double *__restrict__ Xm, int64_t np, int B, int N,
                      int ncb, const int *__restrict__ skip) {
    extern __shared__ double xs[];              // [KR][ncb * 16 + 4]
    if (skip && *skip) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = lane >> 4, pl = lane & 15;
    const int ld = ncb * 16 + 4;
    const int64_t pw = ((int64_t)blockIdx.x * 8 + wave) * 16 * MT;
    d4 acc[MT][MAXC];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int c = 0; c < MAXC; ++c) acc[m][c] = d4{0, 0, 0, 0};
    auto load_a = [&](int k0, d4 (&a)[MT]) {
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int64_t pa = pw + m * 16 + pl;
            a[m] = pa < np ? *(const d4 *)(psi + bidx(np, B, pa, k0 + 4 * j)) : d4{0, 0, 0, 0};
        }
    };
    auto mma = [&](const d4 (&a)[MT], int k16) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = k16 + 4 * j + i;
#pragma unroll
            for (int c = 0; c < MAXC; ++c) {
                if (c < ncb) {
                    const double b = xs[r * ld + c * 16 + pl];
#pragma unroll
                    for (int m = 0; m < MT; ++m)
                        acc[m][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m][i], b, acc[m][c], 0, 0, 0);
                }
            }
        }
    };
    static_assert(KR == 32, "two 16-state blocks per staged slice of X");
    d4 a0[MT], a1[MT];
    load_a(0, a0);
    for (int kc = 0; kc < N; kc += KR) {
        __syncthreads();
        for (int e = threadIdx.x; e < KR * ncb * 16; e += 512) {
            const int r = e / (ncb * 16), col = e % (ncb * 16), k = kc + r;
            xs[r * ld + col] = (k < N && col < N) ? Xm[(int64_t)k * N + col] : 0.0;
        }
        __syncthreads();
        if (kc + 16 < N) load_a(kc + 16, a1);
        mma(a0, 0);
        if (kc + 32 < N) load_a(kc + 32, a0);
        if (kc + 16 < N) mma(a1, 16);
    }
    // every read of this work-group's points is done before the first store
    __syncthreads();
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int c = 0; c < MAXC; ++c) {
            if (c < ncb) {
                const int col = c * 16 + pl;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t p = pw + m * 16 + 4 * r + j;
                    if (p < np && col < N) psi[bidx(np, B, p, col)] = acc[m][c][r];
                }
            }
        }
}

// Persistent form for N <= 128 (the padded X, N16 x (N16 + 4) doubles, fits
// in LDS): one work-group per CU stages X once and walks point tiles of
// 8 * 16 * MT points (tile = blockIdx.x + t * gridDim.x); the A loads of
// the next 16-state block, across tile ends too, are in flight while the
// current block is multiplied.  Each wave reads all N states of its own
// points before it writes them, so the in-place update needs no barrier.
constexpr int kRotPad = 4;    // doubles of padding per LDS row of X
constexpr int kRotXLds = 128 * (128 + kRotPad) * 8;
template <int MT>
__global__ void __launch_bounds__(512)
rotate_f64_px_kernel(double *__restrict__ psi, const double *__restrict__ Xm, int64_t np, int B, int N, int ncb,
                     int64_t ntiles, const int *__restrict__ skip, int upper) {
    constexpr int MAXC = 8;
    extern __shared__ double xs[];              // [N16][ncb * 16 + kRotPad]
    if (skip && *skip) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = lane >> 4, pl = lane & 15;
    const int ld = ncb * 16 + kRotPad;
    for (int e = threadIdx.x; e < ncb * 16 * ncb * 16; e += 512) {
        const int r = e / (ncb * 16), col = e % (ncb * 16);
        xs[r * ld + col] = (r < N && col < N) ? Xm[(int64_t)r * N + col] : 0.0;
    }
    __syncthreads();
    const int nkb = N / 16;                     // 16-state blocks (N is a multiple of B >= 16)
    auto load_a = [&](int64_t tile, int kb, d4 (&a)[MT]) {
        const int64_t pw = (tile * 8 + wave) * 16 * MT;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int64_t pa = pw + m * 16 + pl;
            a[m] = pa < np ? *(const d4 *)(psi + bidx(np, B, pa, 16 * kb + 4 * j)) : d4{0, 0, 0, 0};
        }
    };
    d4 acc[MT][MAXC];
    auto mma = [&](const d4 (&a)[MT], int kb) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * kb + 4 * j + i;
#pragma unroll
            for (int c = 0; c < MAXC; ++c) {
                // upper-triangular X (the inverse Cholesky factor): its
                // 16 x 16 blocks below the diagonal are zero
                if (c < ncb && !(upper && c < kb)) {
                    const double b = xs[r * ld + c * 16 + pl];
#pragma unroll
                    for (int m = 0; m < MT; ++m)
                        acc[m][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m][i], b, acc[m][c], 0, 0, 0);
                }
            }
        }
    };
    int64_t tile = blockIdx.x;
    if (tile >= ntiles) return;
    d4 a0[MT], a1[MT];
    load_a(tile, 0, a0);
    while (true) {
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int c = 0; c < MAXC; ++c) acc[m][c] = d4{0, 0, 0, 0};
        const int64_t next = tile + gridDim.x;
        // blocks in pairs: a0 holds block kb, a1 block kb + 1
        for (int kb = 0; kb < nkb; kb += 2) {
            if (kb + 1 < nkb) load_a(tile, kb + 1, a1);
            mma(a0, kb);
            if (kb + 2 < nkb) load_a(tile, kb + 2, a0);
            else if (next < ntiles) load_a(next, 0, a0);
            if (kb + 1 < nkb) mma(a1, kb + 1);
        }
        const int64_t pw = (tile * 8 + wave) * 16 * MT;
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int c = 0; c < MAXC; ++c) {
                if (c < ncb) {
                    const int col = c * 16 + pl;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t p = pw + m * 16 + 4 * r + j;
                        if (p < np && col < N) psi[bidx(np, B, p, col)] = acc[m][c][r];
                    }
                }
            }
        if (next >= ntiles) break;
        tile = next;
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
// point), B = X (32 states x 16 columns).  The three X terms are staged
// through LDS, 32 rows at a time, shared by the 8 waves of a work-group
// that owns 8 * 16 * MT points and all N <= 16 * MAXC columns (X is read
// once per work-group, not per wave).
constexpr int XLD = 40;    // LDS row of one column: 32 bf16 + 8 pad (80 bytes)
template <int MT, int MAXC>
__global__ void __launch_bounds__(512)
rotate_bf16x3_lds_kernel(float *__restrict__ psi, const unsigned short *__restrict__ xth,
                         const unsigned short *__restrict__ xtl, const unsigned short *__restrict__ xtm,
                         int64_t np, int B, int N, int N32, int ncb, const int *__restrict__ skip) {
    extern __shared__ unsigned short xl[];     // [3][ncb * 16][XLD]
    if (skip && *skip) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ncol = ncb * 16;
    const int64_t pw = ((int64_t)blockIdx.x * 8 + wave) * 16 * MT;
    f4 acc[MT][MAXC];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int c = 0; c < MAXC; ++c) acc[m][c] = f4{0, 0, 0, 0};
    for (int k0 = 0; k0 < N32; k0 += 32) {
        __syncthreads();
        // 16-byte pieces: (term, column, quarter of the 32 rows)
        for (int e = threadIdx.x; e < 3 * ncol * 4; e += 512) {
            const int q = e & 3, col = (e >> 2) % ncol, term = (e >> 2) / ncol;
            const unsigned short *src = term == 0 ? xth : (term == 1 ? xtm : xtl);
            *(us8 *)(xl + (term * ncol + col) * XLD + 8 * q) = *(const us8 *)(src + (int64_t)col * N32 + k0 + 8 * q);
        }
        __syncthreads();
        const int kb = k0 + 8 * (lane / 16);
        bf8 A0[MT], A1[MT], A2[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int64_t pa = pw + m * 16 + lane % 16;
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
            A0[m] = __builtin_bit_cast(bf8, a0);
            A1[m] = __builtin_bit_cast(bf8, a1);
            A2[m] = __builtin_bit_cast(bf8, a2);
        }
#pragma unroll
        for (int c = 0; c < MAXC; ++c) {
            if (c < ncb) {
                const int o = (c * 16 + lane % 16) * XLD + 8 * (lane / 16);
                const bf8 X0 = __builtin_bit_cast(bf8, *(const us8 *)(xl + o));
                const bf8 X1 = __builtin_bit_cast(bf8, *(const us8 *)(xl + ncol * XLD + o));
                const bf8 X2 = __builtin_bit_cast(bf8, *(const us8 *)(xl + 2 * ncol * XLD + o));
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    // smallest terms first
                    acc[m][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A2[m], X0, acc[m][c], 0, 0, 0);
                    acc[m][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1[m], X1, acc[m][c], 0, 0, 0);
                    acc[m][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0[m], X2, acc[m][c], 0, 0, 0);
                    acc[m][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1[m], X0, acc[m][c], 0, 0, 0);
                    acc[m][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0[m], X1, acc[m][c], 0, 0, 0);
                    acc[m][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0[m], X0, acc[m][c], 0, 0, 0);
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int c = 0; c < MAXC; ++c) {
            if (c < ncb) {
                const int col = c * 16 + lane % 16;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t p = pw + m * 16 + 4 * (lane / 16) + r;
                    if (p < np && col < N) psi[bidx(np, B, p, col)] = acc[m][c][r];
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

// Persistent BF16x3 rotation for N32 <= 128 and B a multiple of 8: one
// work-group per CU holds the three X terms of every 32-row slice in LDS
// ([slice][term][column][XLD]) and walks point tiles; a lane's 8 states of
// one point are two 16-byte loads, and the next slice's (or tile's) loads
// are in flight while the current slice is multiplied.  The splitting of
// psi and the order of the six products are those of the kernel above.
constexpr int kRotBfLds = 4 * 3 * 128 * XLD * 2;
template <int MT>
__global__ void __launch_bounds__(512)
rotate_bf16x3_px_kernel(float *__restrict__ psi, const unsigned short *__restrict__ xth,
                        const unsigned short *__restrict__ xtl, const unsigned short *__restrict__ xtm,
                        int64_t np, int B, int N, int N32, int ncb, int64_t ntiles, const int *__restrict__ skip) {
    constexpr int MAXC = 8;
    extern __shared__ unsigned short xl[];
    if (skip && *skip) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ncol = ncb * 16, nsl = N32 / 32;
    for (int e = threadIdx.x; e < nsl * 3 * ncol * 4; e += 512) {
        const int q = e & 3, col = (e >> 2) % ncol, rest = (e >> 2) / ncol;
        const int term = rest % 3, sl = rest / 3;
        const unsigned short *src = term == 0 ? xth : (term == 1 ? xtm : xtl);
        *(us8 *)(xl + ((sl * 3 + term) * ncol + col) * XLD + 8 * q) =
            *(const us8 *)(src + (int64_t)col * N32 + sl * 32 + 8 * q);
    }
    __syncthreads();
    auto load_a = [&](int64_t tile, int sl, f4 (&a)[MT][2]) {
        const int64_t pw = (tile * 8 + wave) * 16 * MT;
        const int kb = sl * 32 + 8 * (lane / 16);
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int64_t pa = pw + m * 16 + lane % 16;
            if (pa < np && kb < N) {
                const float *src = psi + bidx(np, B, pa, kb);
                a[m][0] = *(const f4 *)src;
                a[m][1] = *(const f4 *)(src + 4);
            } else {
                a[m][0] = f4{0, 0, 0, 0};
                a[m][1] = f4{0, 0, 0, 0};
            }
        }
    };
    f4 acc[MT][MAXC];
    auto mma = [&](const f4 (&a)[MT][2], int sl) {
        bf8 A0[MT], A1[MT], A2[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            us8 a0, a1, a2;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const float v = a[m][t >> 2][t & 3];
                const unsigned short h0 = bf16_rne(v);
                const float r1 = v - bf16_to_f(h0);
                const unsigned short h1 = bf16_rne(r1);
                a0[t] = h0;
                a1[t] = h1;
                a2[t] = bf16_rne(r1 - bf16_to_f(h1));
            }
            A0[m] = __builtin_bit_cast(bf8, a0);
            A1[m] = __builtin_bit_cast(bf8, a1);
            A2[m] = __builtin_bit_cast(bf8, a2);
        }
        const unsigned short *xs = xl + sl * 3 * ncol * XLD;
#pragma unroll
        for (int c = 0; c < MAXC; ++c) {
            if (c < ncb) {
                const int o = (c * 16 + lane % 16) * XLD + 8 * (lane / 16);
                const bf8 X0 = __builtin_bit_cast(bf8, *(const us8 *)(xs + o));
                const bf8 X1 = __builtin_bit_cast(bf8, *(const us8 *)(xs + ncol * XLD + o));
                const bf8 X2 = __builtin_bit_cast(bf8, *(const us8 *)(xs + 2 * ncol * XLD + o));
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    acc[m][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A2[m], X0, acc[m][c], 0, 0, 0);
                    acc[m][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1[m], X1, acc[m][c], 0, 0, 0);
                    acc[m][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0[m], X2, acc[m][c], 0, 0, 0);
                    acc[m][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1[m], X0, acc[m][c], 0, 0, 0);
                    acc[m][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0[m], X1, acc[m][c], 0, 0, 0);
                    acc[m][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0[m], X0, acc[m][c], 0, 0, 0);
                }
            }
        }
    };
    int64_t tile = blockIdx.x;
    if (tile >= ntiles) return;
    f4 a0[MT][2], a1[MT][2];
    load_a(tile, 0, a0);
    while (true) {
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int c = 0; c < MAXC; ++c) acc[m][c] = f4{0, 0, 0, 0};
        const int64_t next = tile + gridDim.x;
        for (int sl = 0; sl < nsl; sl += 2) {
            if (sl + 1 < nsl) load_a(tile, sl + 1, a1);
            mma(a0, sl);
            if (sl + 2 < nsl) load_a(tile, sl + 2, a0);
            else if (next < ntiles) load_a(next, 0, a0);
            if (sl + 1 < nsl) mma(a1, sl + 1);
        }
        const int64_t pw = (tile * 8 + wave) * 16 * MT;
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int c = 0; c < MAXC; ++c) {
                if (c < ncb) {
                    const int col = c * 16 + lane % 16;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t p = pw + m * 16 + 4 * (lane / 16) + r;
                        if (p < np && col < N) psi[bidx(np, B, p, col)] = acc[m][c][r];
                    }
                }
            }
        if (next >= ntiles) break;
        tile = next;
    }
}

// ------------------------------------------------------------- Cholesky
// S = U^T U, U upper with positive diagonal (right-looking, one work-group;
// the working copy W lives in LDS when it fits, else in global memory).
// Thread (c, g) owns the columns j = c (mod 128) and the rows i = g (mod
// nt/128) of the trailing update, so no index is divided.  Step k reads only
// row k of W (unscaled: the update subtracts W[k][i] W[k][j] / d) and writes
// only rows below it, so a step needs one barrier; row k of U goes straight
// to U.  Every thread reads the same pivot d, so all leave the loop together
// on a bad pivot.  info = 0, or the 1-based column whose pivot is not
// positive (that row of U and all after it stay zero).
template <bool LDSW>
__global__ void __launch_bounds__(1024)
cholesky_kernel(const double *__restrict__ S, double *__restrict__ Wg, double *__restrict__ U, int N,
                int *__restrict__ info) {
    extern __shared__ double ldsW[];
    double *W = LDSW ? ldsW : Wg;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int c = tid & 127, g = tid >> 7, ng = nt >> 7;
    for (int e = tid; e < N * N; e += nt) {
        W[e] = S[e];
        U[e] = 0.0;
    }
    __syncthreads();
    int bad = 0;
    for (int k = 0; k < N; ++k) {
        const double d = W[k * N + k];
        if (!(d > 0.0) || !isfinite(d)) {
            bad = k + 1;
            break;
        }
        const double piv = sqrt(d), inv = 1.0 / piv, invd = 1.0 / d;
        for (int j = c; j < N; j += 128) {
            if (j < k) continue;
            const double wkj = W[k * N + j];
            if (g == 0) U[k * N + j] = j == k ? piv : wkj * inv;
            const double f = wkj * invd;
            for (int i = k + 1 + g; i <= j; i += ng) W[i * N + j] -= W[k * N + i] * f;
        }
        __syncthreads();
    }
    if (tid == 0) *info = bad;
}

// Inverse of an upper-triangular U: one wave per column j solves U t = e_j
// by back substitution.  T = U^-1 is upper triangular.  Skipped when
// info != 0.
//  - LDSU (N <= 128): column-oriented.  U^T is staged in LDS; lane l keeps
//    the running sums s_m = sum_(k > m) U[m][k] t_k of rows m = l, l + 64;
//    for k = j down to 0, t_k = -s_k / U[k][k] (t_j = 1 / U[j][j]) is read
//    from the lane that owns row k, and every lane adds U[m][k] t_k to its
//    rows m < k.  Each step is one broadcast instead of a wave reduction;
//    the sums run in a fixed order (k descending).
//  - otherwise: row-oriented, the inner products split over the 64 lanes
//    and summed in a fixed butterfly, U read from global memory.
constexpr size_t kTrinvLds = 128 * 128 * sizeof(double);
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
template <bool LDSU>
__global__ void __launch_bounds__(1024)
trinv_kernel(const double *__restrict__ U, double *__restrict__ T, int N, const int *__restrict__ info) {
    extern __shared__ double ut[];              // LDSU: U^T [N][N]
    __shared__ double cols[LDSU ? 1 : 16 * 256];
    if (*info) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if constexpr (LDSU) {
        for (int e = threadIdx.x; e < N * N; e += blockDim.x) ut[(e % N) * N + e / N] = U[e];
        __syncthreads();
        for (int j = wave; j < N; j += nw) {
            double s0 = 0.0, s1 = 0.0, t0 = 0.0, t1 = 0.0;
            for (int k = j; k >= 0; --k) {
                const double sk = readlane_f64(k < 64 ? s0 : s1, k & 63);
                const double ukk = ut[k * N + k];
                const double tk = k == j ? 1.0 / ukk : -sk / ukk;
                if (lane == (k & 63)) {
                    if (k < 64) t0 = tk;
                    else t1 = tk;
                }
                if (lane < k) s0 += ut[k * N + lane] * tk;
                if (lane + 64 < k) s1 += ut[k * N + lane + 64] * tk;
            }
            if (lane < N) T[lane * N + j] = lane <= j ? t0 : 0.0;
            if (lane + 64 < N) T[(lane + 64) * N + j] = lane + 64 <= j ? t1 : 0.0;
        }
    } else {
        double *t = cols + wave * 256;
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
}

// ------------------------------------------------------ Jacobi eigensolver
// Cyclic parallel Jacobi on a symmetric A (N <= 256, FP64, one work-group).
// Each round rotates N/2 disjoint pairs (round-robin ordering) as
// A <- J^T A J, V <- V J; sweeps repeat until the off-diagonal norm is below
// tol * ||A||_F or max_sweeps is reached.  A lives in LDS when it fits
// (LDSA), else in global memory.  Eigenvalues ascending; each eigenvector's
// largest-magnitude component is made positive.
// Cyclic Jacobi in the parallel (round-robin) ordering: each round
// annihilates M/2 disjoint pivots (p, q) at once, so A <- J^T A J splits
// into independent 2x2 blocks (pair k) x (pair l).  One work-group; A lives
// in LDS with an odd row stride when it fits, else in place in global
// memory.  A must be symmetric; only blocks k <= l are computed and the
// transposed block is mirrored, keeping A exactly symmetric.  The rotations
// (c, s) are recorded per round for the eigenvector kernel; the final
// diagonal goes to diag.
template <bool LDSA>
__global__ void __launch_bounds__(1024)
jacobi_rot_kernel(double *__restrict__ Ag, int N, int max_sweeps, double tol, int *__restrict__ sweeps_out,
                  double2 *__restrict__ rot, double *__restrict__ diag) {
    extern __shared__ double ldsA[];
    // a pair's indices and rotation, each one LDS access for the updates
    __shared__ int2 pq[128];
    __shared__ double2 csn[128];
    __shared__ double red[16];
    __shared__ int stop;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    const int ld = LDSA ? N + 1 : N;
    double *A = LDSA ? ldsA : Ag;
    if (LDSA)
        for (int i = wave; i < N; i += nw)
            for (int j = lane; j < N; j += 64) A[i * ld + j] = Ag[i * N + j];
    const int M = N + (N & 1);        // even number of players (a dummy when N is odd)
    const int h = M / 2;
    // N <= 128: rounds keep only the upper triangle up to date (each element
    // written once, at (min, max) of its indices); larger N: both
    const bool upper = h <= 64 && nw == 16;
    __syncthreads();
    // Frobenius norms (all entries, then off-diagonal) in a fixed order
    auto block_sum = [&](bool offdiag) {
        double loc = 0.0;
        for (int i = wave; i < N; i += nw)
            for (int j = lane; j < N; j += 64) {
                const double a = A[i * ld + j];
                if (upper && offdiag) loc += j > i ? 2.0 * (a * a) : 0.0;
                else if (!offdiag || i != j) loc += a * a;
            }
        loc = wave_sum(loc);
        if (lane == 0) red[wave] = loc;
        __syncthreads();
        double t = 0.0;
        for (int w2 = 0; w2 < nw; ++w2) t += red[w2];
        __syncthreads();
        return t;
    };
    const double fro = sqrt(block_sum(false));
    // N <= 128: rows a = P and h - 1 - P of the upper triangle of 2x2 blocks
    // hold h + 1 blocks together, so wave w takes the row pairs P = w and
    // w + 16 (one block per lane each, the 65th on lanes 0 and 1): at most
    // three blocks (k, l) per lane, the same in every round
    int kl[3][2];
    bool on[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int P = j < 2 ? wave + 16 * j : wave + 16 * lane;
        const int c = j < 2 ? lane : 64;
        const int a = P, b = h - 1 - P;
        const int na = h - a, nt = a < b ? h + 1 : na;
        on[j] = upper && a <= b && c < nt && (j < 2 || lane < 2);
        kl[j][0] = c < na ? a : b;
        kl[j][1] = c < na ? a + c : b + (c - na);
    }
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        const double off = sqrt(block_sum(true));
        if (tid == 0) stop = !(off > tol * fro);
        __syncthreads();
        if (stop) break;
        for (int r = 0; r < M - 1; ++r) {
            for (int k = tid; k < h; k += blockDim.x) {
                auto pos = [&](int i) {
                    if (i == 0) return 0;
                    int x = i - 1 + r;               // < 2 (M - 1)
                    if (x >= M - 1) x -= M - 1;
                    return x + 1;
                };
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
                pq[k] = make_int2(p, q);
                csn[k] = make_double2(c, s);
                rot[((int64_t)sweep * (M - 1) + r) * h + k] = make_double2(c, s);
            }
            __syncthreads();
            if (upper) {
                // a round reads and writes each element of the upper triangle
                // once (element (a, b) at (min, max)), and only the blocks'
                // own elements, so all blocks are loaded before any is
                // stored (the loads of a round then overlap in LDS)
                auto cix = [&](int a, int b) { return a < b ? a * ld + b : b * ld + a; };
                double x[3][4];
                int4 ix[3];
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    if (!on[j]) continue;
                    const int2 u = pq[kl[j][0]], v = pq[kl[j][1]];
                    const int pk = u.x, qk = u.y, pl = v.x, ql = v.y;
                    ix[j] = make_int4(pk, qk, pl, ql);
                    x[j][0] = A[cix(pk, pl)];
                    x[j][1] = ql < N ? A[cix(pk, ql)] : 0.0;
                    x[j][2] = qk < N ? A[cix(qk, pl)] : 0.0;
                    x[j][3] = qk < N && ql < N ? A[cix(qk, ql)] : 0.0;
                }
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    if (!on[j]) continue;
                    const int k = kl[j][0], l = kl[j][1];
                    const int pk = ix[j].x, qk = ix[j].y, pl = ix[j].z, ql = ix[j].w;
                    const bool vk = qk < N, vl = ql < N;
                    const double2 rk = csn[k], rl = csn[l];
                    const double ck = rk.x, sk = rk.y, cl = rl.x, sl = rl.y;
                    const double x00 = x[j][0], x01 = x[j][1], x10 = x[j][2], x11 = x[j][3];
                    const double y00 = cl * x00 - sl * x01, y01 = sl * x00 + cl * x01;
                    const double y10 = cl * x10 - sl * x11, y11 = sl * x10 + cl * x11;
                    const double z00 = ck * y00 - sk * y10, z01 = ck * y01 - sk * y11;
                    const double z10 = sk * y00 + ck * y10, z11 = sk * y01 + ck * y11;
                    if (l == k) {
                        A[pk * ld + pk] = z00;
                        if (vk) {
                            A[cix(pk, qk)] = 0.0;
                            A[qk * ld + qk] = z11;
                        }
                        continue;
                    }
                    A[cix(pk, pl)] = z00;
                    if (vl) A[cix(pk, ql)] = z01;
                    if (vk) A[cix(qk, pl)] = z10;
                    if (vk && vl) A[cix(qk, ql)] = z11;
                }
                __syncthreads();
                continue;
            }
            for (int k = wave; k < h; k += nw) {
                const int pk = pq[k].x, qk = pq[k].y;
                const bool vk = qk < N;
                const double ck = csn[k].x, sk = csn[k].y;
                for (int l = k + lane; l < h; l += 64) {
                    const int pl = pq[l].x, ql = pq[l].y;
                    const bool vl = ql < N;
                    const double cl = csn[l].x, sl = csn[l].y;
                    const double x00 = A[pk * ld + pl];
                    const double x01 = vl ? A[pk * ld + ql] : 0.0;
                    const double x10 = vk ? A[qk * ld + pl] : 0.0;
                    const double x11 = vk && vl ? A[qk * ld + ql] : 0.0;
                    // columns (A J), then rows (J^T A J)
                    const double y00 = cl * x00 - sl * x01, y01 = sl * x00 + cl * x01;
                    const double y10 = cl * x10 - sl * x11, y11 = sl * x10 + cl * x11;
                    const double z00 = ck * y00 - sk * y10, z01 = ck * y01 - sk * y11;
                    const double z10 = sk * y00 + ck * y10, z11 = sk * y01 + ck * y11;
                    if (l == k) {
                        // the pivot block: off-diagonal annihilated exactly
                        A[pk * ld + pk] = z00;
                        if (vk) {
                            A[pk * ld + qk] = 0.0;
                            A[qk * ld + pk] = 0.0;
                            A[qk * ld + qk] = z11;
                        }
                        continue;
                    }
                    A[pk * ld + pl] = z00;
                    A[pl * ld + pk] = z00;
                    if (vl) {
                        A[pk * ld + ql] = z01;
                        A[ql * ld + pk] = z01;
                    }
                    if (vk) {
                        A[qk * ld + pl] = z10;
                        A[pl * ld + qk] = z10;
                    }
                    if (vk && vl) {
                        A[qk * ld + ql] = z11;
                        A[ql * ld + qk] = z11;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < N; i += blockDim.x) diag[i] = A[i * ld + i];
    if (tid == 0) *sweeps_out = sweep;
}

// Eigenvectors from the recorded rotations: V = J_1 J_2 ... J_R, and the
// rows of V are independent (v <- v J per round), so one wave owns one row
// in LDS and applies every round in order; rotations are staged through LDS
// in groups of 16 rounds.
constexpr int kRotStage = 16;
__global__ void __launch_bounds__(256)
jacobi_vec_kernel(const double2 *__restrict__ rot, const int *__restrict__ sweeps, int N, double *__restrict__ Vw) {
    __shared__ double row[4][256];
    __shared__ double2 stage[kRotStage][128];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i = blockIdx.x * 4 + wave;
    const int M = N + (N & 1), h = M / 2;
    const int R = *sweeps * (M - 1);
    if (i < N)
        for (int j = lane; j < N; j += 64) row[wave][j] = i == j ? 1.0 : 0.0;
    for (int r0 = 0; r0 < R; r0 += kRotStage) {
        const int nr = min(kRotStage, R - r0);
        __syncthreads();
        for (int e = tid; e < nr * h; e += blockDim.x) stage[e / h][e % h] = rot[(int64_t)r0 * h + e];
        __syncthreads();
        if (i >= N) continue;
        for (int t = 0; t < nr; ++t) {
            const int r = (r0 + t) % (M - 1);
            for (int k = lane; k < h; k += 64) {
                auto pos = [&](int x) { return x == 0 ? 0 : ((x - 1 + r) % (M - 1)) + 1; };
                int p = pos(k), q = pos(M - 1 - k);
                if (p > q) { const int tt = p; p = q; q = tt; }
                if (q >= N) continue;
                const double c = stage[t][k].x, s = stage[t][k].y;
                const double vp = row[wave][p], vq = row[wave][q];
                row[wave][p] = c * vp - s * vq;
                row[wave][q] = s * vp + c * vq;
            }
            // the next round reads entries other lanes of this wave wrote
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    if (i < N)
        for (int j = lane; j < N; j += 64) Vw[(int64_t)i * N + j] = row[wave][j];
}

// Sort ascending (rank by value, ties by index) and normalise each
// eigenvector's sign so that its largest-magnitude entry is positive
// (ties: the lowest index); one wave per eigenvector.
__global__ void __launch_bounds__(1024)
jacobi_sort_kernel(const double *__restrict__ diag, const double *__restrict__ Vw, int N, double *__restrict__ V,
                   double *__restrict__ evals) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int j = wave; j < N; j += nw) {
        const double d = diag[j];
        int rank = 0;
        double big = -1.0;
        int arg = 0;
        for (int i = lane; i < N; i += 64) {
            const double e = diag[i];
            rank += (e < d) || (e == d && i < j);
            const double v = fabs(Vw[(int64_t)i * N + j]);
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
        const double sg = Vw[(int64_t)arg * N + j] < 0 ? -1.0 : 1.0;
        for (int i = lane; i < N; i += 64) V[(int64_t)i * N + rank] = sg * Vw[(int64_t)i * N + j];
    }
}

// Padded states (index >= n of an N x N matrix): identity on their
// diagonal, so Cholesky and the eigensolver leave them untouched.
// S[j][k] = <x_j|y_k> for complex states from the real products of their
// parts: (re re + im im) + i (re im' - im re').
__global__ void complex_fold_kernel(const double *__restrict__ G, double *__restrict__ S, int N) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)N * N) return;
    const int j = (int)(e / N), k = (int)(e % N);
    const int64_t M = 2 * (int64_t)N;
    const double *r0 = G + (2 * j) * M, *r1 = G + (2 * j + 1) * M;
    S[2 * e] = r0[2 * k] + r1[2 * k + 1];
    S[2 * e + 1] = r0[2 * k + 1] - r1[2 * k];
}

__global__ void pad_identity_kernel(double *__restrict__ S, int N, int n) {
    const int i = n + blockIdx.x * 256 + threadIdx.x;
    if (i < N) S[(int64_t)i * N + i] = 1.0;
}

// Leading n x n block of an N x N matrix, compacted to stride n.
__global__ void compact_kernel(const double *__restrict__ A, int N, int n, double *__restrict__ Ac) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n * n) return;
    Ac[e] = A[(int64_t)(e / n) * N + e % n];
}

// V (N x N) = diag(Vc (n x n), identity); evals beyond n set to zero.
__global__ void expand_kernel(const double *__restrict__ Vc, int n, int N, double *__restrict__ V,
                              double *__restrict__ evals) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= N * N) return;
    const int i = e / N, j = e % N;
    V[e] = (i < n && j < n) ? Vc[i * n + j] : (i == j ? 1.0 : 0.0);
    if (e >= n && e < N) evals[e] = 0.0;
}

}  // namespace

// 16 x 16 output blocks of an N16 x N16 product: all of them (full), and
// those with row block <= column block in row order (symmetric product).
__global__ void gram_blocks_kernel(int nb16, int2 *__restrict__ full, int2 *__restrict__ syrk) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= nb16 * nb16) return;
    const int i = t / nb16, j = t % nb16;
    full[t] = int2{i, j};
    if (i <= j) syrk[i * nb16 - i * (i - 1) / 2 + (j - i)] = int2{i, j};
}

// ------------------------------------------------------------ launchers
rs_status gram(DenseWork &w, const void *X, const void *Y, int64_t np, int B, int nblk, int dtype,
               int prec, double dv, double *S, int mode, hipStream_t st) {
    const int N16 = (nblk * B + 15) / 16 * 16;
    GramScratch ws{w.partial.as<double>(), (int64_t)w.partial.bytes, w.red.as<double>(), w.d_blocks_full.as<int2>(),
                   w.d_blocks_syrk.as<int2>(), w.max_chunks};
    rs_status e = gram_core(ws, w.blocks_n != N16, X, Y, np, B, nblk, dtype, prec, dv, S, mode, st);
    if (!e) w.blocks_n = N16;
    return e;
}

// Sum of the chunk partials into S (reduce mode as in gram_reduce2_kernel).
static rs_status gram_reduce(const GramScratch &w, int nchunks, int N, int N16, int rmode, double dv, double *S,
                             hipStream_t st) {
    const int64_t ne = (int64_t)N16 * N16;
    const int ng = std::min(kRedGroups, nchunks);
    const int cpg = (nchunks + ng - 1) / ng;
    hipLaunchKernelGGL(gram_reduce1_kernel, dim3((unsigned)((ne + 255) / 256), ng), dim3(256), 0, st, w.partial,
                       nchunks, cpg, ne, w.red);
    RS_HIP(hipGetLastError());
    hipLaunchKernelGGL(gram_reduce2_kernel, dim3((N * N + 255) / 256), dim3(256), 0, st, w.red, ng, N, N16, rmode,
                       dv, S);
    RS_HIP(hipGetLastError());
    return RS_OK;
}

rs_status gram_core(const GramScratch &w, bool make_lists, const void *X, const void *Y, int64_t np, int B,
                    int nblk, int dtype, int prec, double dv, double *S, int mode, hipStream_t st) {
    const int N = nblk * B;
    const int N16 = (N + 15) / 16 * 16;
    const bool syrk = X == Y;
    const int nb16 = N16 / 16;
    if (make_lists) {
        hipLaunchKernelGGL(gram_blocks_kernel, dim3((nb16 * nb16 + 255) / 256), dim3(256), 0, st, nb16,
                           w.blocks_full, w.blocks_syrk);
        RS_HIP(hipGetLastError());
    }
    const int nblocks = syrk ? nb16 * (nb16 + 1) / 2 : nb16 * nb16;
    const int2 *dbl = syrk ? w.blocks_syrk : w.blocks_full;
    const int per_wg = 4 * MAXB;
    const int nsplit = (nblocks + per_wg - 1) / per_wg;
    const int bps = (nblocks + nsplit - 1) / nsplit;
    const bool bf = dtype == RS_F32 && prec == RS_PREC_BF16X3;
    if (bf && B == 32 && N == 128) {
        // about two waves per SIMD: 512 chunks of four waves (symmetric) or
        // 256 of eight, in whole 32-point k-steps, bounded by the workspace
        const int64_t want = syrk ? 512 : 256;
        int64_t CP = std::max<int64_t>((np + want - 1) / want, (np + w.max_chunks - 1) / w.max_chunks);
        CP = std::max<int64_t>(32, (CP + 31) / 32 * 32);
        const int nchunks = (int)((np + CP - 1) / CP);
        if ((int64_t)nchunks * 128 * 128 * (int64_t)sizeof(double) > w.partial_bytes)
            return fail(RS_EINVAL, "gram: workspace too small");
        if (CP * 128 > INT32_MAX) return fail(RS_EINVAL, "gram: chunk too large for 32-bit offsets");
        if (syrk)
            hipLaunchKernelGGL(gram_bf_r32_kernel<true>, dim3(nchunks), dim3(256), 0, st, (const float *)X,
                               (const float *)Y, np, CP, w.partial);
        else
            hipLaunchKernelGGL(gram_bf_r32_kernel<false>, dim3(nchunks), dim3(512), 0, st, (const float *)X,
                               (const float *)Y, np, CP, w.partial);
        RS_HIP(hipGetLastError());
        return gram_reduce(w, nchunks, N, N16, syrk ? 3 : mode, dv, S, st);
    }
    if (dtype == RS_F64 && B == 32 && N == 128) {
        // about two waves per SIMD: 1024 chunks of two waves (symmetric) or
        // 512 of four, each a whole number of load groups of 4 * kGramDepth
        // points, bounded by the partial-sum workspace
        const int64_t group = 4 * kGramDepth;
        int64_t CP = std::max<int64_t>((np + (syrk ? 1023 : 511)) / (syrk ? 1024 : 512),
                                       (np + w.max_chunks - 1) / w.max_chunks);
        CP = std::max<int64_t>(group, (CP + group - 1) / group * group);
        const int nchunks = (int)((np + CP - 1) / CP);
        if ((int64_t)nchunks * 128 * 128 * (int64_t)sizeof(double) > w.partial_bytes)
            return fail(RS_EINVAL, "gram: workspace too small");
        if (CP * 256 > INT32_MAX) return fail(RS_EINVAL, "gram: chunk too large for 32-bit offsets");
        if (syrk)
            hipLaunchKernelGGL(gram_f64_r32_kernel<true>, dim3(nchunks), dim3(128), 0, st, (const double *)X,
                               (const double *)Y, np, CP, w.partial);
        else
            hipLaunchKernelGGL(gram_f64_r32_kernel<false>, dim3(nchunks), dim3(256), 0, st, (const double *)X,
                               (const double *)Y, np, CP, w.partial);
        RS_HIP(hipGetLastError());
        return gram_reduce(w, nchunks, N, N16, syrk ? 3 : mode, dv, S, st);
    }
    // small chunks: several work-groups per compute unit (each owns all
    // output blocks of its chunk), bounded by the partial-sum workspace
    int64_t CP = bf ? 1024 : 512;
    while ((np + CP - 1) / CP > w.max_chunks) CP *= 2;
    if (CP > (1 << 30)) return fail(RS_EINVAL, "gram: grid too large for the partial-sum workspace");
    const int nchunks = (int)((np + CP - 1) / CP);
    if ((int64_t)nchunks * N16 * N16 * (int64_t)sizeof(double) > w.partial_bytes)
        return fail(RS_EINVAL, "gram: workspace too small");
    dim3 grid(nchunks, nsplit);
    if (dtype == RS_F64) {
        const size_t lds = (syrk ? 1 : 2) * (size_t)KC64 * N16 * sizeof(double);
        // exact per-wave share: every work-group holds bps = 4 * nbw blocks
        const int nbw = (bps % 4 == 0 && nblocks % bps == 0) ? bps / 4 : 0;
#define RS_GRAM64(S, NB)                                                                                  \
    hipLaunchKernelGGL((gram_f64_kernel<S, NB>), grid, dim3(256), lds, st, (const double *)X, (const double *)Y, \
                       np, B, N, N16, (int)CP, dbl, nblocks, bps, w.partial)
        // (the interleaved form is faster at 9 blocks per wave, the symmetric
        // product of 128 states; at 16 its 128 accumulators cost occupancy)
        if (nbw == 9) {
            if (syrk) RS_GRAM64(true, 9);
            else RS_GRAM64(false, 9);
        } else {
            if (syrk) RS_GRAM64(true, 0);
            else RS_GRAM64(false, 0);
        }
#undef RS_GRAM64
    } else if (bf) {
        const size_t lds = (syrk ? 2 : 4) * (size_t)N16 * LDSROW * sizeof(unsigned short);
#define RS_GRAMBF(S, V)                                                                                   \
    hipLaunchKernelGGL((gram_bf16x3_kernel<S, V>), grid, dim3(256), lds, st, (const float *)X, (const float *)Y, \
                       np, B, N, N16, (int)CP, dbl, nblocks, bps, w.partial)
        if (B % 4 == 0) {
            if (syrk) RS_GRAMBF(true, true);
            else RS_GRAMBF(false, true);
        } else {
            if (syrk) RS_GRAMBF(true, false);
            else RS_GRAMBF(false, false);
        }
#undef RS_GRAMBF
    } else {
        return fail(RS_ENOTSUP, "gram: FP32 data needs RS_PREC_BF16X3");
    }
    RS_HIP(hipGetLastError());
    return gram_reduce(w, nchunks, N, N16, syrk ? 1 : mode, dv, S, st);
}

rs_status rotate(DenseWork &w, void *psi, const double *Xm, int64_t np, int B, int nblk, int dtype, int prec,
                 const int *skip, hipStream_t st, bool upper) {
    const int N = nblk * B;
    const int N16 = (N + 15) / 16 * 16;
    const int ncb = N16 / 16;
    if (dtype == RS_F64) {
        const size_t lds = (size_t)KR * (ncb * 16 + 4) * sizeof(double);
        if (B % 16 == 0 && ncb <= 8) {
            // X resident in LDS, one persistent work-group per CU
            if (!w.rot_lds_set) {
                RS_HIP(hipFuncSetAttribute((const void *)rotate_f64_px_kernel<kRotMT>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, kRotXLds));
                int dev = 0;
                RS_HIP(hipGetDevice(&dev));
                RS_HIP(hipDeviceGetAttribute(&w.ncu, hipDeviceAttributeMultiprocessorCount, dev));
                w.rot_lds_set = true;
            }
            const int64_t ntiles = (np + 128 * kRotMT - 1) / (128 * kRotMT);
            const size_t xl = (size_t)N16 * (N16 + kRotPad) * sizeof(double);
            const unsigned grid = (unsigned)std::min<int64_t>(ntiles, std::max(w.ncu, 1));
            hipLaunchKernelGGL((rotate_f64_px_kernel<kRotMT>), dim3(grid), dim3(512), xl, st, (double *)psi, Xm, np,
                               B, N, ncb, ntiles, skip, upper ? 1 : 0);
        } else if (B % 16 == 0) {
            // ncb > 8 here: the persistent kernel above takes the rest
            hipLaunchKernelGGL((rotate_f64_vec_kernel<1, MAXC64>), dim3((unsigned)((np + 127) / 128)), dim3(512),
                               lds, st, (double *)psi, Xm, np, B, N, ncb, skip);
        } else if (ncb <= 8) {
            const unsigned g2 = (unsigned)((np + 255) / 256);
            hipLaunchKernelGGL((rotate_f64_lds_kernel<2, 8>), dim3(g2), dim3(512), lds, st, (double *)psi, Xm, np, B, N,
                               ncb, skip);
        } else {
            const unsigned g1 = (unsigned)((np + 127) / 128);
            hipLaunchKernelGGL((rotate_f64_lds_kernel<1, MAXC64>), dim3(g1), dim3(512), lds, st, (double *)psi, Xm, np, B, N,
                               ncb, skip);
        }
    } else if (prec == RS_PREC_BF16X3) {
        const int N32 = (N + 31) / 32 * 32;
        hipLaunchKernelGGL(split_xt_kernel, dim3((N16 * N32 + 255) / 256), dim3(256), 0, st, Xm, N, N16, N32,
                           w.xth.as<unsigned short>(), w.xtl.as<unsigned short>(), w.xtm.as<unsigned short>());
        RS_HIP(hipGetLastError());
        const size_t lds = (size_t)3 * ncb * 16 * XLD * sizeof(unsigned short);
        if (B % 8 == 0 && ncb <= 8 && N32 <= 128) {
            // all slices of X resident in LDS, one persistent work-group per CU
            if (!w.rotbf_lds_set) {
                RS_HIP(hipFuncSetAttribute((const void *)rotate_bf16x3_px_kernel<2>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, kRotBfLds));
                int dev = 0;
                RS_HIP(hipGetDevice(&dev));
                RS_HIP(hipDeviceGetAttribute(&w.ncu, hipDeviceAttributeMultiprocessorCount, dev));
                w.rotbf_lds_set = true;
            }
            const int64_t ntiles = (np + 255) / 256;
            const size_t xlb = (size_t)(N32 / 32) * 3 * ncb * 16 * XLD * sizeof(unsigned short);
            const unsigned grid = (unsigned)std::min<int64_t>(ntiles, std::max(w.ncu, 1));
            hipLaunchKernelGGL((rotate_bf16x3_px_kernel<2>), dim3(grid), dim3(512), xlb, st, (float *)psi,
                               w.xth.as<unsigned short>(), w.xtl.as<unsigned short>(), w.xtm.as<unsigned short>(), np,
                               B, N, N32, ncb, ntiles, skip);
        } else if (ncb <= 8)
            hipLaunchKernelGGL((rotate_bf16x3_lds_kernel<2, 8>), dim3((unsigned)((np + 255) / 256)), dim3(512), lds,
                               st, (float *)psi, w.xth.as<unsigned short>(), w.xtl.as<unsigned short>(),
                               w.xtm.as<unsigned short>(), np, B, N, N32, ncb, skip);
        else
            hipLaunchKernelGGL((rotate_bf16x3_lds_kernel<1, MAXC64>), dim3((unsigned)((np + 127) / 128)), dim3(512),
                               lds, st, (float *)psi, w.xth.as<unsigned short>(), w.xtl.as<unsigned short>(),
                               w.xtm.as<unsigned short>(), np, B, N, N32, ncb, skip);
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
    if (N <= 128) {
        RS_HIP(hipFuncSetAttribute((const void *)trinv_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)kTrinvLds));
        const size_t lds = (size_t)N * N * sizeof(double);
        hipLaunchKernelGGL(trinv_kernel<true>, dim3(1), dim3(1024), lds, st, U, T, N, info_dev);
    } else {
        hipLaunchKernelGGL(trinv_kernel<false>, dim3(1), dim3(1024), 0, st, U, T, N, info_dev);
    }
    RS_HIP(hipGetLastError());
    return RS_OK;
}

rs_status eigh(DenseWork &w, double *A, double *V, double *evals, int N, hipStream_t st, int max_sweeps) {
    max_sweeps = std::max(0, std::min(max_sweeps, kMaxSweeps));
    const size_t lds = (size_t)N * (N + 1) * sizeof(double);
    double *diag = w.diag.as<double>();
    double2 *rot = w.rot.as<double2>();
    if (lds <= kJacobiLds) {
        if (!w.jacobi_lds_set) {
            RS_HIP(hipFuncSetAttribute((const void *)jacobi_rot_kernel<true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kJacobiLds));
            w.jacobi_lds_set = true;
        }
        hipLaunchKernelGGL(jacobi_rot_kernel<true>, dim3(1), dim3(1024), lds, st, A, N, max_sweeps, 1e-15,
                           w.sweeps.as<int>(), rot, diag);
    } else {
        hipLaunchKernelGGL(jacobi_rot_kernel<false>, dim3(1), dim3(1024), 0, st, A, N, max_sweeps, 1e-15,
                           w.sweeps.as<int>(), rot, diag);
    }
    RS_HIP(hipGetLastError());
    hipLaunchKernelGGL(jacobi_vec_kernel, dim3((N + 3) / 4), dim3(256), 0, st, rot, w.sweeps.as<int>(), N,
                       w.mwork.as<double>());
    RS_HIP(hipGetLastError());
    hipLaunchKernelGGL(jacobi_sort_kernel, dim3(1), dim3(1024), 0, st, diag, w.mwork.as<double>(), N, V, evals);
    RS_HIP(hipGetLastError());
    return RS_OK;
}

rs_status dense_work_init(DenseWork &w, int64_t np, int max_states) {
    const int N16 = (max_states + 15) / 16 * 16;
    const int N32 = (max_states + 31) / 32 * 32;
    w.max_states = max_states;
    // chunk partials: at most 256 MiB
    w.max_chunks = (int)std::max<int64_t>(64, std::min<int64_t>(4096, ((int64_t)256 << 20) / ((int64_t)N16 * N16 * 8)));
    rs_status s = RS_OK;
    const size_t nb16 = (size_t)(N16 / 16) * (N16 / 16);
    if (!s) s = w.partial.alloc((size_t)w.max_chunks * N16 * N16 * sizeof(double));
    if (!s) s = w.red.alloc((size_t)kRedGroups * N16 * N16 * sizeof(double));
    if (!s) s = w.d_blocks_syrk.alloc(nb16 * sizeof(int2));
    if (!s) s = w.d_blocks_full.alloc(nb16 * sizeof(int2));
    if (!s) s = w.mwork.alloc((size_t)max_states * max_states * sizeof(double));
    if (!s) s = w.xth.alloc((size_t)N16 * N32 * sizeof(unsigned short));
    if (!s) s = w.xtl.alloc((size_t)N16 * N32 * sizeof(unsigned short));
    if (!s) s = w.xtm.alloc((size_t)N16 * N32 * sizeof(unsigned short));
    if (!s) s = w.sweeps.alloc(sizeof(int));
    if (!s) s = w.diag.alloc((size_t)max_states * sizeof(double));
    const size_t M = max_states + (max_states & 1);
    if (!s) s = w.rot.alloc((size_t)kMaxSweeps * (M - 1) * (M / 2) * sizeof(double2));
    (void)np;
    return s;
}

}  // namespace rs

namespace rs {

rs_status complex_fold(const double *G, double *S, int N, hipStream_t st) {
    const int64_t n2 = (int64_t)N * N;
    hipLaunchKernelGGL(complex_fold_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, G, S, N);
    RS_HIP(hipGetLastError());
    return RS_OK;
}

rs_status pad_identity(double *S, int N, int n, hipStream_t st) {
    if (n >= N) return RS_OK;
    hipLaunchKernelGGL(pad_identity_kernel, dim3((N - n + 255) / 256), dim3(256), 0, st, S, N, n);
    RS_HIP(hipGetLastError());
    return RS_OK;
}

rs_status eigh_leading(DenseWork &w, double *A, double *V, double *evals, int N, int n, double *scratch_a,
                       double *scratch_v, hipStream_t st, int max_sweeps) {
    if (n >= N) return eigh(w, A, V, evals, N, st, max_sweeps);
    hipLaunchKernelGGL(compact_kernel, dim3((n * n + 255) / 256), dim3(256), 0, st, A, N, n, scratch_a);
    RS_HIP(hipGetLastError());
    rs_status e = eigh(w, scratch_a, scratch_v, evals, n, st, max_sweeps);
    if (e) return e;
    hipLaunchKernelGGL(expand_kernel, dim3((N * N + 255) / 256), dim3(256), 0, st, scratch_v, n, N, V, evals);
    RS_HIP(hipGetLastError());
    return RS_OK;
}

}  // namespace rs


// ------------------------------------------------- overlap without allocation
// rs_overlap_noalloc runs the same point-summed product as rs_overlap, with
// its chunk partials, group sums and block lists in `scratch`, a fixed device
// array that the code object holds on every GPU the library runs on, so the
// call allocates nothing.  In host code `scratch` names a host-side stand-in:
// its device address comes from hipGetSymbolAddress, once per device, and
// only that address is handed to kernels.
#include <mutex>

namespace {

constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;   // 64 MiB per GPU
constexpr int kNoallocMaxStates = 256;
constexpr size_t kNoallocListBytes = 4096;                   // both block lists
__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call made with that device current).
rs_status noalloc_scratch(unsigned char **out) {
    int dev = 0;
    RS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return rs::fail(RS_EINVAL, "rs_overlap_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return rs::hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return rs::fail(RS_EHIP, "rs_overlap_noalloc: no device address for the scratch array");
        g_scratch_dev[dev] = p;
    }
    *out = (unsigned char *)g_scratch_dev[dev];
    return RS_OK;
}

}  // namespace

extern "C" rs_status rs_overlap_noalloc(const rs_grid *g, const void *x, const void *y, double *S, int32_t nblk,
                                        int32_t B, int32_t dtype, int32_t prec, void *stream) {
    using rs::fail;
    if (!g || !x || !y || !S) return fail(RS_EINVAL, "rs_overlap_noalloc: null argument");
    if (g->host_only) return fail(RS_EINVAL, "rs_overlap_noalloc: host-only grid");
    if (B < 1 || B > 64 || (B & (B - 1))) return fail(RS_EINVAL, "rs_overlap_noalloc: B must be a power of two in [1, 64]");
    if (nblk < 1 || (int64_t)nblk * B > kNoallocMaxStates)
        return fail(RS_EINVAL, "rs_overlap_noalloc: nblk*B must be in [1, 256] (the fixed scratch holds the partial "
                               "sums of at most 256 states)");
    if (dtype == RS_F64 && prec != RS_PREC_NATIVE)
        return fail(RS_ENOTSUP, "rs_overlap_noalloc: FP64 fields use RS_PREC_NATIVE contractions");
    if (dtype == RS_F32 && prec != RS_PREC_BF16X3)
        return fail(RS_ENOTSUP, "rs_overlap_noalloc: FP32 fields use RS_PREC_BF16X3 contractions");
    if (dtype != RS_F64 && dtype != RS_F32) return fail(RS_EINVAL, "rs_overlap_noalloc: bad dtype");
    unsigned char *base = nullptr;
    rs_status st = noalloc_scratch(&base);
    if (st) return st;
    const int64_t N16 = ((int64_t)nblk * B + 15) / 16 * 16;
    const int64_t mat = N16 * N16 * (int64_t)sizeof(double);
    const int64_t red_bytes = rs::kGramRedGroups * mat;
    const int64_t part_off = (int64_t)kNoallocListBytes + red_bytes;
    const int64_t part_bytes = (int64_t)kNoallocScratchBytes - part_off;
    rs::GramScratch ws;
    ws.blocks_full = (int2 *)base;
    ws.blocks_syrk = (int2 *)(base + kNoallocListBytes / 2);
    ws.red = (double *)(base + kNoallocListBytes);
    ws.partial = (double *)(base + part_off);
    ws.partial_bytes = part_bytes;
    ws.max_chunks = (int)(part_bytes / mat);
    const double dv = g->h * g->h * g->h;
    // the block lists are rebuilt on every call: the previous call on this
    // GPU may have had another N
    return rs::gram_core(ws, true, x, y, g->np, B, nblk, dtype, prec, dv, S, 0, (hipStream_t)stream);
}
