// Per-state reductions over grid points for fields in the block layout
// [nblk][np][B]: sums with FP64 accumulation, per chunk of points, then a
// fixed-order sum over the chunks (deterministic, independent of timing).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace rsred {
namespace {

constexpr int kChunk = 2048;  // points per reduction chunk

// partial[k][chunk][col], col = blk * B + s.  One work-group per (chunk,
// block); lanes: state s, rows r striding over the chunk's points.  With a
// block map, grid row y covers block bmap[y] (the other blocks' partial
// sums are left as they are).
template <int K, typename Op>
__global__ void __launch_bounds__(256)
colreduce_kernel(Op op, int64_t np, int B, int nchunks, int N, double *__restrict__ partial,
                 const int *__restrict__ bmap) {
    __shared__ double red[K][256];
    const int blk = bmap ? bmap[blockIdx.y] : (int)blockIdx.y, tid = threadIdx.x;
    const int s = tid % B, r = tid / B, R = 256 / B;
    const int64_t p0 = (int64_t)blockIdx.x * kChunk, p1 = min<int64_t>(np, p0 + kChunk);
    const int col = blk * B + s;
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    // unrolled so that several points' loads are in flight per thread
#pragma unroll 4
    for (int64_t p = p0 + r; p < p1; p += R) op((int64_t)blk * np * B + p * B + s, col, acc);
#pragma unroll
    for (int k = 0; k < K; ++k) red[k][tid] = acc[k];
    __syncthreads();
    for (int st = R / 2; st > 0; st >>= 1) {
        if (r < st)
#pragma unroll
            for (int k = 0; k < K; ++k) red[k][tid] += red[k][tid + st * B];
        __syncthreads();
    }
    if (r == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) partial[((int64_t)k * nchunks + blockIdx.x) * N + col] = red[k][s];
}

// One wave per output: lanes sum strided chunks, then a fixed butterfly.
__global__ void __launch_bounds__(256)
colreduce_final(const double *__restrict__ partial, int K, int nchunks, int N, double dv, double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int idx = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (idx >= K * N) return;
    const int k = idx / N, c = idx % N;
    double s = 0.0;
    for (int ch = lane; ch < nchunks; ch += 64) s += partial[((int64_t)k * nchunks + ch) * N + c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) out[idx] = dv * s;
}

// Sums for all nblk * B columns; with bmap (device, nmap entries) only the
// listed blocks are reduced this time and the other columns' outputs repeat
// whatever their partial sums last held.
template <int K, typename Op>
rs_status colreduce(const Op &op, int64_t np, int B, int nblk, double dv, double *partial, double *out,
                    hipStream_t st, const int *bmap = nullptr, int nmap = 0) {
    const int N = nblk * B;
    const int nchunks = (int)((np + kChunk - 1) / kChunk);
    hipLaunchKernelGGL((colreduce_kernel<K, Op>), dim3(nchunks, bmap ? nmap : nblk), dim3(256), 0, st, op, np, B,
                       nchunks, N, partial, bmap);
    RS_HIP(hipGetLastError());
    hipLaunchKernelGGL(colreduce_final, dim3((K * N + 3) / 4), dim3(256), 0, st, partial, K, nchunks, N, dv,
                       out);
    RS_HIP(hipGetLastError());
    return RS_OK;
}

}  // namespace
}  // namespace rsred
