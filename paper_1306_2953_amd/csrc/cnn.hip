// Learned preconditioner for the RMM-DIIS step, and the shifted-kinetic
// solves that produce its training targets.
//
// The paper leaves the eigensolver's preconditioner open (Sec. 3 uses a
// filter); this is the project's learned replacement.  Network f: three
// 3x3x3 cross-correlation layers without bias, channels 1 -> 8 -> 8 -> 1,
// tanh after the first two, every layer's output zeroed off the domain.
// Preconditioner: K(r) = s g(sigma) f(r / s), s the rms of r over the grid
// points, g = softplus(a + b log(-sigma h^2)).  Targets: x = (T - sigma)^-1 r
// by conjugate gradients with the 25-point kinetic stencil (Sec. 5.1).
//
// Network fields are dense boxes, channels last: [n][Z][Y][X][C], FP32.  On
// a grid the box is the smallest axis-aligned box holding every point, zero
// outside the domain (periodic grids wrap).  Parameters are one FP32 vector:
// w1 [8][1][27], w2 [8][8][27], w3 [1][8][27] (tap t = 9 dz + 3 dy + dx,
// input offset (dx-1, dy-1, dz-1)), then a, b.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "colreduce.hpp"
#include "internal.hpp"

namespace rs {
rs_status kinetic_apply(const rs_grid *g, const void *psi, void *out, int nblk, int B, int dtype,
                        hipStream_t st);
}

namespace {
using namespace rsred;

constexpr int kW1 = 0, kW2 = 216, kW3 = 1944, kNW = 2160, kNP = 2162;
constexpr int kWgPts = 2048;   // points per work-group in the weight gradients

__device__ __forceinline__ int wrap_or_flag(int v, int n, bool wrap, bool &ok) {
    if (wrap) return v < 0 ? v + n : (v >= n ? v - n : v);
    ok = ok && v >= 0 && v < n;
    return v;
}

// ------------------------------------------------------------ convolution
// MODE 0: out = mask * tanh(conv(in));  MODE 1: out = mask * conv(in);
// MODE 2: out = mask * conv(in) * (1 - act^2)  (backward through tanh).
// W [CO][CI][27]; taps outside the box are zero (or wrap).  A work-group
// owns a TZ x TY x TX block of outputs of one box: it stages the block and
// its one-point border, channels last, in LDS once, then each thread
// computes two x-neighbouring outputs from there, which share the loads of
// their taps.  Per output the sum runs over taps t = 9 dz + 3 dy + dx, then
// output channel, then input channel, one fused multiply-add each; the
// weights are uniform across the work-group.
constexpr int kTX = 16, kTY = 8, kTZ = 4;   // 512 outputs per work-group, 2 per thread

template <int CI, int CO, int MODE>
__global__ void __launch_bounds__(256)
conv_kernel(const float *__restrict__ in, float *__restrict__ out, const float *__restrict__ W,
            const float *__restrict__ act, const int32_t *__restrict__ boxpt, int n, int Z, int Y, int X,
            int wrap, int ntx, int nty, int ntz) {
    constexpr int HX = kTX + 2, HY = kTY + 2, HZ = kTZ + 2;
    __shared__ __attribute__((aligned(16))) float tile[HZ * HY * HX * CI];
    const int bid = blockIdx.x;
    const int tx = bid % ntx, ty = (bid / ntx) % nty, tz = (bid / (ntx * nty)) % ntz;
    const int img = bid / (ntx * nty * ntz);
    const int x0 = tx * kTX, y0 = ty * kTY, z0 = tz * kTZ;
    const int vol = Z * Y * X;
    const float *base = in + (int64_t)img * vol * CI;
    // stage the block and its border; positions more than one point past the
    // box feed only outputs that are not computed and are left zero
    for (int e = threadIdx.x; e < HZ * HY * HX; e += 256) {
        const int hx = e % HX, hy = (e / HX) % HY, hz = e / (HX * HY);
        const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
        bool ok = gx <= X && gy <= Y && gz <= Z;
        const int xx = wrap_or_flag(gx, X, wrap, ok);
        const int yy = wrap_or_flag(gy, Y, wrap, ok);
        const int zz = wrap_or_flag(gz, Z, wrap, ok);
        ok = ok && xx >= 0 && xx < X && yy >= 0 && yy < Y && zz >= 0 && zz < Z;
        float *dst = tile + e * CI;
        if constexpr (CI == 8) {
            float4 lo = make_float4(0.f, 0.f, 0.f, 0.f), hi = lo;
            if (ok) {
                const float *src = base + ((int64_t)(zz * Y + yy) * X + xx) * CI;
                lo = *(const float4 *)src;
                hi = *(const float4 *)(src + 4);
            }
            *(float4 *)dst = lo;
            *(float4 *)(dst + 4) = hi;
        } else {
#pragma unroll
            for (int c = 0; c < CI; ++c) dst[c] = ok ? base[((int64_t)(zz * Y + yy) * X + xx) * CI + c] : 0.f;
        }
    }
    __syncthreads();
    const int t = threadIdx.x;
    const int lx = 2 * (t % (kTX / 2)), ly = (t / (kTX / 2)) % kTY, lz = t / (kTX / 2 * kTY);
    float acc0[CO], acc1[CO];
#pragma unroll
    for (int c = 0; c < CO; ++c) acc0[c] = acc1[c] = 0.f;
    // (dz, dy) stays a loop: unrolled, the loads of all nine rows would be
    // hoisted and the work-group would run at one wave per SIMD
#pragma unroll 1
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll 1
        for (int dy = 0; dy < 3; ++dy) {
            // border coordinates: output lx sits at lx + 1, tap dx reads lx + dx
            const float *row = tile + (((lz + dz) * HY + (ly + dy)) * HX + lx) * CI;
            float v[4][CI];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if constexpr (CI == 8) {
                    const float4 lo = *(const float4 *)(row + j * CI), hi = *(const float4 *)(row + j * CI + 4);
                    v[j][0] = lo.x; v[j][1] = lo.y; v[j][2] = lo.z; v[j][3] = lo.w;
                    v[j][4] = hi.x; v[j][5] = hi.y; v[j][6] = hi.z; v[j][7] = hi.w;
                } else {
#pragma unroll
                    for (int c = 0; c < CI; ++c) v[j][c] = row[j * CI + c];
                }
            }
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int tap = 9 * dz + 3 * dy + dx;
#pragma unroll
                for (int co = 0; co < CO; ++co)
#pragma unroll
                    for (int ci = 0; ci < CI; ++ci) {
                        const float w = W[(co * CI + ci) * 27 + tap];
                        acc0[co] = fmaf(w, v[dx][ci], acc0[co]);
                        acc1[co] = fmaf(w, v[dx + 1][ci], acc1[co]);
                    }
            }
        }
    const int y = y0 + ly, z = z0 + lz;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int x = x0 + lx + k;
        if (x >= X || y >= Y || z >= Z) continue;
        const int q = (z * Y + y) * X + x;
        const int64_t gid = (int64_t)img * vol + q;
        const bool inside = boxpt == nullptr || boxpt[q] >= 0;
        float *dst = out + gid * CO;
        float r[CO];
#pragma unroll
        for (int c = 0; c < CO; ++c) {
            const float a = k == 0 ? acc0[c] : acc1[c];
            float o;
            if constexpr (MODE == 0) o = tanhf(a);
            else if constexpr (MODE == 1) o = a;
            else {
                const float ac = act[gid * CO + c];
                o = a * (1.f - ac * ac);
            }
            r[c] = inside ? o : 0.f;
        }
        if constexpr (CO == 8) {
            *(float4 *)dst = make_float4(r[0], r[1], r[2], r[3]);
            *(float4 *)(dst + 4) = make_float4(r[4], r[5], r[6], r[7]);
        } else {
#pragma unroll
            for (int c = 0; c < CO; ++c) dst[c] = r[c];
        }
    }
}

// Launches conv_kernel over n boxes of Z x Y x X points.
template <int CI, int CO, int MODE>
void conv(const float *in, float *out, const float *W, const float *act, const int32_t *boxpt, int n, int Z, int Y,
          int X, int wrap, hipStream_t st) {
    const int ntx = (X + kTX - 1) / kTX, nty = (Y + kTY - 1) / kTY, ntz = (Z + kTZ - 1) / kTZ;
    const int64_t nwg = (int64_t)ntx * nty * ntz * n;
    hipLaunchKernelGGL((conv_kernel<CI, CO, MODE>), dim3((unsigned)nwg), dim3(256), 0, st, in, out, W, act, boxpt, n,
                       Z, Y, X, wrap, ntx, nty, ntz);
}

// Layer 2 of the forward pass (8 -> 8 channels, tanh) on the matrix cores:
// per row of 16 outputs an implicit GEMM D[point][co] = sum over k = (tap,
// ci) of A[point][k] W[co][ci][tap], K = 27 taps x 8 channels in 7 chunks of
// 32 (4 taps each; the 28th tap gets zero weights), N = the 8 channels of a
// 16-wide tile.  Inputs and weights are split as hi + lo bfloat16 (the
// input block once per work-group, into hi and lo planes in LDS) and the
// four products lo.lo + hi.lo + lo.hi + hi.hi are summed in FP32 on
// mfma_f32_16x16x32_bf16, which keeps FP32 accuracy.  Lane l supplies A row
// l % 16 (point x0 + l % 16) and B column l % 16 (channel), both for k =
// 8 (l / 16) .. + 7 (tap 4 c + l / 16 of chunk c, channels 0..7), and
// receives D rows 4 (l / 16) + r, r < 4, of column l % 16.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// bfloat16 with round-to-nearest-even (finite inputs)
__device__ __forceinline__ unsigned short bf16_rne(float x) {
    const uint32_t u = __builtin_bit_cast(uint32_t, x);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

__global__ void __launch_bounds__(256)
conv2_mfma_kernel(const float *__restrict__ in, float *__restrict__ out, const float *__restrict__ W,
                  const int32_t *__restrict__ boxpt, int n, int Z, int Y, int X, int wrap, int ntx, int nty,
                  int ntz) {
    constexpr int HX = kTX + 2, HY = kTY + 2, HZ = kTZ + 2, NH = HX * HY * HZ;
    __shared__ __attribute__((aligned(16))) unsigned short th[NH * 8], tl[NH * 8];
    const int vol = Z * Y * X;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // this lane's B operands (channel co, taps 4 c + g of the 7 chunks) and
    // the LDS offsets of its A operands relative to the row's first point,
    // once for all the tiles this work-group takes
    const int co = lane % 16, g = lane / 16;
    bf8 bh[7], bl[7];
    int aoff[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) {
        const int tap = 4 * c + g;
        us8 h, l;
#pragma unroll
        for (int ci = 0; ci < 8; ++ci) {
            const float w = co < 8 && tap < 27 ? W[(co * 8 + ci) * 27 + tap] : 0.f;
            h[ci] = bf16_rne(w);
            l[ci] = bf16_rne(w - bf16_to_f(h[ci]));
        }
        bh[c] = __builtin_bit_cast(bf8, h);
        bl[c] = __builtin_bit_cast(bf8, l);
        const int t = min(tap, 26);   // the 28th tap: zero weights, any finite input
        aoff[c] = (((t / 9) * HY + (t / 3) % 3) * HX + t % 3 + co) * 8;
    }
    const int ntile = ntx * nty * ntz * n;
    for (int bid = blockIdx.x; bid < ntile; bid += gridDim.x) {
        const int tx = bid % ntx, ty = (bid / ntx) % nty, tz = (bid / (ntx * nty)) % ntz;
        const int img = bid / (ntx * nty * ntz);
        const int x0 = tx * kTX, y0 = ty * kTY, z0 = tz * kTZ;
        const float *base = in + (int64_t)img * vol * 8;
        __syncthreads();   // the previous tile's reads of the LDS block are done
        for (int e = tid; e < NH; e += 256) {
            const int hx = e % HX, hy = (e / HX) % HY, hz = e / (HX * HY);
            const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
            bool ok = gx <= X && gy <= Y && gz <= Z;
            const int xx = wrap_or_flag(gx, X, wrap, ok);
            const int yy = wrap_or_flag(gy, Y, wrap, ok);
            const int zz = wrap_or_flag(gz, Z, wrap, ok);
            ok = ok && xx >= 0 && xx < X && yy >= 0 && yy < Y && zz >= 0 && zz < Z;
            float v[8];
            if (ok) {
                const float *src = base + ((int64_t)(zz * Y + yy) * X + xx) * 8;
                const float4 a = *(const float4 *)src, b = *(const float4 *)(src + 4);
                v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
            } else {
#pragma unroll
                for (int c = 0; c < 8; ++c) v[c] = 0.f;
            }
            us8 h, l;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                h[c] = bf16_rne(v[c]);
                l[c] = bf16_rne(v[c] - bf16_to_f(h[c]));
            }
            *(us8 *)(th + e * 8) = h;
            *(us8 *)(tl + e * 8) = l;
        }
        __syncthreads();
        for (int row = wave; row < kTZ * kTY; row += 4) {
            const int lz = row / kTY, ly = row % kTY;
            const int rb = (lz * HY + ly) * HX * 8;
            // one accumulator per product: four independent chains
            f4 acc[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[k] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int c = 0; c < 7; ++c) {
                const bf8 ah = __builtin_bit_cast(bf8, *(const us8 *)(th + rb + aoff[c]));
                const bf8 al = __builtin_bit_cast(bf8, *(const us8 *)(tl + rb + aoff[c]));
                acc[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bl[c], acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[c], acc[1], 0, 0, 0);
                acc[2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[c], acc[2], 0, 0, 0);
                acc[3] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[c], acc[3], 0, 0, 0);
            }
            // the small products first; lanes of channels 0..7 hold the 4
            // outputs of rows 4 g .. 4 g + 3, and hand the last two to the
            // lane 8 above (whose channel column is empty), so every lane
            // evaluates two tanh
            const f4 d = ((acc[0] + acc[1]) + acc[2]) + acc[3];
            const float s0 = __shfl_xor(d[2], 8, 64), s1 = __shfl_xor(d[3], 8, 64);
            const int cc = co & 7, r0 = co < 8 ? 0 : 2;
            const float v0 = co < 8 ? d[0] : s0, v1 = co < 8 ? d[1] : s1;
            const int y = y0 + ly, z = z0 + lz;
            if (y >= Y || z >= Z) continue;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int x = x0 + 4 * g + r0 + k;
                if (x >= X) continue;
                const int q = (z * Y + y) * X + x;
                const bool inside = boxpt == nullptr || boxpt[q] >= 0;
                out[((int64_t)img * vol + q) * 8 + cc] = inside ? tanhf(k == 0 ? v0 : v1) : 0.f;
            }
        }
    }
}

// Weights of the input adjoint: Wt[ci][co][26 - t] = W[co][ci][t].
__global__ void flip_kernel(const float *__restrict__ params, float *__restrict__ wt) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kNW) return;
    int off, CI, CO;
    if (i < kW2) { off = kW1; CI = 1; CO = 8; }
    else if (i < kW3) { off = kW2; CI = 8; CO = 8; }
    else { off = kW3; CI = 8; CO = 1; }
    const int j = i - off, t = j % 27, ci = (j / 27) % CI, co = j / (27 * CI);
    wt[off + (ci * CO + co) * 27 + (26 - t)] = params[i];
}

// Weight gradient partials: partial[wg][co][ci][t] = sum over the
// work-group's points p of d[p][co] x[p + off(t)][ci].
template <int CI, int CO>
__global__ void __launch_bounds__(256)
wgrad_kernel(const float *__restrict__ xin, const float *__restrict__ d, int n, int Z, int Y, int X, int wrap,
             float *__restrict__ partial) {
    __shared__ float dl[64][CO];
    __shared__ int pc[64][4];
    const int tid = threadIdx.x;
    const bool act = tid < 27 * CI;
    const int t = tid / CI, ci = tid % CI;
    const int ddz = t / 9 - 1, ddy = (t / 3) % 3 - 1, ddx = t % 3 - 1;
    const int vol = Z * Y * X, total = vol * n;
    const int p0 = blockIdx.x * kWgPts, p1 = min(total, p0 + kWgPts);
    float acc[CO];
#pragma unroll
    for (int c = 0; c < CO; ++c) acc[c] = 0.f;
    for (int pb = p0; pb < p1; pb += 64) {
        const int cnt = min(64, p1 - pb);
        __syncthreads();
        for (int e = tid; e < cnt * CO; e += 256) dl[e / CO][e % CO] = d[(int64_t)pb * CO + e];
        if (tid < cnt) {
            const int p = pb + tid, img = p / vol, q = p - img * vol;
            pc[tid][0] = img;
            pc[tid][1] = q % X;
            pc[tid][2] = (q / X) % Y;
            pc[tid][3] = q / (X * Y);
        }
        __syncthreads();
        if (!act) continue;
        for (int j = 0; j < cnt; ++j) {
            bool ok = true;
            const int xx = wrap_or_flag(pc[j][1] + ddx, X, wrap, ok);
            const int yy = wrap_or_flag(pc[j][2] + ddy, Y, wrap, ok);
            const int zz = wrap_or_flag(pc[j][3] + ddz, Z, wrap, ok);
            if (!ok) continue;
            const float xv = xin[((int64_t)pc[j][0] * vol + (zz * Y + yy) * X + xx) * CI + ci];
#pragma unroll
            for (int c = 0; c < CO; ++c) acc[c] = fmaf(xv, dl[j][c], acc[c]);
        }
    }
    if (act)
#pragma unroll
        for (int c = 0; c < CO; ++c) partial[(int64_t)blockIdx.x * (CO * CI * 27) + (c * CI + ci) * 27 + t] = acc[c];
}

// grad[off + j] = sum over work-groups of partial[wg][j] (FP64, fixed order;
// one wave per entry).
__global__ void __launch_bounds__(256)
wgrad_final(const float *__restrict__ partial, int nwg, int nw, float *__restrict__ grad) {
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= nw) return;
    double s = 0.0;
    for (int w = lane; w < nwg; w += 64) s += partial[(int64_t)w * nw + j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) grad[j] = (float)s;
}

__device__ double softplus_d(double z) { return z > 0 ? z + log1p(exp(-z)) : log1p(exp(z)); }
__device__ double sigmoid_d(double z) { return 0.5 * (1.0 + tanh(0.5 * z)); }

// g_i = softplus(a + b l_i), l_i = log(-sigma_i h^2); gz = [g, z, l] per sample.
__global__ void gain_kernel(const float *__restrict__ params, const double *__restrict__ sigma, double h, int n,
                            double *__restrict__ gz) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double l = log(-sigma[i] * h * h);
    const double z = (double)params[kNW] + (double)params[kNW + 1] * l;
    gz[3 * i] = softplus_d(z);
    gz[3 * i + 1] = z;
    gz[3 * i + 2] = l;
}

__device__ __forceinline__ bool interior(int q, int Z, int Y, int X, int margin) {
    const int x = q % X, y = (q / X) % Y, z = q / (X * Y);
    return !(x < margin || y < margin || z < margin || x >= X - margin || y >= Y - margin || z >= Z - margin);
}

// em = M (g f - t), tm = M t (M: points at least `margin` from the faces).
__global__ void err_kernel(const float *__restrict__ f, const float *__restrict__ t, const double *__restrict__ gz,
                           int Z, int Y, int X, int margin, int n, float *__restrict__ em, float *__restrict__ tm) {
    const int vol = Z * Y * X;
    const int gid = blockIdx.x * 256 + threadIdx.x;
    if (gid >= vol * n) return;
    const int i = gid / vol, q = gid - i * vol;
    const bool in = interior(q, Z, Y, X, margin);
    em[gid] = in ? (float)(gz[3 * i] * (double)f[gid] - (double)t[gid]) : 0.f;
    tm[gid] = in ? t[gid] : 0.f;
}

// out = (T - sigma_i) x on each box, zero outside: the 25-point star of
// Sec. 5.1 in first-difference form.
__global__ void kin_kernel(const float *__restrict__ x, float *__restrict__ out, const double *__restrict__ sigma,
                           double h, int Z, int Y, int X, int n) {
    const int vol = Z * Y * X;
    const int gid = blockIdx.x * 256 + threadIdx.x;
    if (gid >= vol * n) return;
    const int i = gid / vol, q = gid - i * vol;
    const int cx = q % X, cy = (q / X) % Y, cz = q / (X * Y);
    const float *b = x + (int64_t)i * vol;
    const float c[5] = {0.f, 8.f / 5.f, -1.f / 5.f, 8.f / 315.f, -1.f / 560.f};
    const float v = b[q];
    float acc = 0.f;
#pragma unroll
    for (int m = 1; m <= 4; ++m) {
        const float xm = cx - m >= 0 ? b[q - m] : 0.f, xp = cx + m < X ? b[q + m] : 0.f;
        const float ym = cy - m >= 0 ? b[q - m * X] : 0.f, yp = cy + m < Y ? b[q + m * X] : 0.f;
        const float zm = cz - m >= 0 ? b[q - m * X * Y] : 0.f, zp = cz + m < Z ? b[q + m * X * Y] : 0.f;
        acc += c[m] * (((xm - v) + (xp - v)) + ((ym - v) + (yp - v)) + ((zm - v) + (zp - v)));
    }
    out[gid] = (float)(-0.5 / (h * h) * (double)acc - sigma[i] * (double)v);
}

// Per (chunk, sample) sums: <em|A em>, <tm|A tm>, <M f|A em>.
__global__ void __launch_bounds__(256)
loss_partial_kernel(const float *__restrict__ em, const float *__restrict__ ae, const float *__restrict__ tm,
                    const float *__restrict__ at, const float *__restrict__ f, int Z, int Y, int X, int margin,
                    int nch, double *__restrict__ partial) {
    __shared__ double red[3][256];
    const int i = blockIdx.y, tid = threadIdx.x;
    const int vol = Z * Y * X, per = (vol + nch - 1) / nch;
    const int q0 = blockIdx.x * per, q1 = min(vol, q0 + per);
    double a0 = 0, a1 = 0, a2 = 0;
    for (int q = q0 + tid; q < q1; q += 256) {
        const int64_t k = (int64_t)i * vol + q;
        const double aev = ae[k];
        a0 += (double)em[k] * aev;
        a1 += (double)tm[k] * (double)at[k];
        if (interior(q, Z, Y, X, margin)) a2 += (double)f[k] * aev;
    }
    red[0][tid] = a0;
    red[1][tid] = a1;
    red[2][tid] = a2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s)
            for (int k = 0; k < 3; ++k) red[k][tid] += red[k][tid + s];
        __syncthreads();
    }
    if (tid < 3) partial[((int64_t)i * nch + blockIdx.x) * 3 + tid] = red[tid][0];
}

// loss = sum_i <e|Ae>_i / sum_i <t|At>_i; coef = 2 / sum_i <t|At>_i (so
// dL/dpred = coef M A e); gain-parameter gradient into grad[kNW], grad[kNW + 1].
__global__ void loss_final_kernel(const double *__restrict__ partial, int n, int nch, const double *__restrict__ gz,
                                  double *__restrict__ coef, double *__restrict__ loss, float *__restrict__ grad) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double E2 = 0, T2 = 0;
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < nch; ++c) {
            E2 += partial[((int64_t)i * nch + c) * 3];
            T2 += partial[((int64_t)i * nch + c) * 3 + 1];
        }
    const double cf = T2 > 0 ? 2.0 / T2 : 0.0;
    double ga = 0, gb = 0;
    for (int i = 0; i < n; ++i) {
        double ef = 0;
        for (int c = 0; c < nch; ++c) ef += partial[((int64_t)i * nch + c) * 3 + 2];
        coef[i] = cf;
        const double dg = cf * ef;
        const double sg = sigmoid_d(gz[3 * i + 1]);
        ga += dg * sg;
        gb += dg * sg * gz[3 * i + 2];
    }
    *loss = T2 > 0 ? E2 / T2 : 0.0;
    grad[kNW] = (float)ga;
    grad[kNW + 1] = (float)gb;
}

__global__ void df_kernel(const float *__restrict__ ae, const double *__restrict__ gz,
                          const double *__restrict__ coef, int Z, int Y, int X, int margin, int n,
                          float *__restrict__ df) {
    const int vol = Z * Y * X;
    const int gid = blockIdx.x * 256 + threadIdx.x;
    if (gid >= vol * n) return;
    const int i = gid / vol, q = gid - i * vol;
    df[gid] = interior(q, Z, Y, X, margin) ? (float)(gz[3 * i] * coef[i] * (double)ae[gid]) : 0.f;
}

// Adam (Kingma and Ba, 2015): c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kNP) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------- grid <-> dense boxes
// Transposing copies through LDS: a work-group moves 64 consecutive box
// points (or grid points) of the B states of one block.
template <typename T>
__global__ void __launch_bounds__(256)
scatter_kernel(const T *__restrict__ r, const int32_t *__restrict__ boxpt, const double *__restrict__ scale,
               int k0, int B, int64_t np, int vol, float *__restrict__ u) {
    __shared__ float tile[64][65];
    const int blk = blockIdx.y, tid = threadIdx.x;
    const int q0 = blockIdx.x * 64;
    const int kb = k0 + blk * B;               // first state of the block
    for (int e = tid; e < 64 * B; e += 256) {
        const int qi = e / B, s = e % B, q = q0 + qi;
        float v = 0.f;
        if (q < vol) {
            const int pt = boxpt[q];
            if (pt >= 0) v = (float)((double)r[((int64_t)(kb / B) * np + pt) * B + s] * scale[kb + s]);
        }
        tile[s][qi] = v;
    }
    __syncthreads();
    for (int e = tid; e < 64 * B; e += 256) {
        const int s = e / 64, qi = e % 64, q = q0 + qi;
        if (q < vol) u[(int64_t)(blk * B + s) * vol + q] = tile[s][qi];
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
gather_kernel(const float *__restrict__ f, const int32_t *__restrict__ boxidx, const double *__restrict__ scale,
              int k0, int B, int64_t np, int vol, T *__restrict__ out) {
    __shared__ float tile[64][65];
    const int blk = blockIdx.y, tid = threadIdx.x;
    const int64_t p0 = (int64_t)blockIdx.x * 64;
    const int kb = k0 + blk * B;
    for (int e = tid; e < 64 * B; e += 256) {
        const int s = e / 64, pi = e % 64;
        const int64_t p = p0 + pi;
        tile[s][pi] = p < np ? f[(int64_t)(blk * B + s) * vol + boxidx[p]] : 0.f;
    }
    __syncthreads();
    for (int e = tid; e < 64 * B; e += 256) {
        const int pi = e / B, s = e % B;
        const int64_t p = p0 + pi;
        if (p < np) out[((int64_t)(kb / B) * np + p) * B + s] = (T)((double)tile[s][pi] * scale[kb + s]);
    }
}

// Crops: u[c][z][y][x] = r(point at box origin + (x, y, z)) * inv_s[state],
// t likewise from x; zero off the domain (or beyond the box unless periodic).
template <typename T>
__global__ void __launch_bounds__(256)
crop_kernel(const T *__restrict__ r, const T *__restrict__ xs, const int32_t *__restrict__ boxpt,
            const int32_t *__restrict__ desc, const double *__restrict__ inv_s, int B, int64_t np, int BZ, int BY,
            int BX, int wrap, int CZ, int CY, int CX, int ncrops, float *__restrict__ u, float *__restrict__ t) {
    const int cvol = CZ * CY * CX;
    const int gid = blockIdx.x * 256 + threadIdx.x;
    if (gid >= cvol * ncrops) return;
    const int c = gid / cvol, q = gid - c * cvol;
    const int k = desc[4 * c];
    bool ok = true;
    const int x = wrap_or_flag(desc[4 * c + 1] + q % CX, BX, wrap, ok);
    const int y = wrap_or_flag(desc[4 * c + 2] + (q / CX) % CY, BY, wrap, ok);
    const int z = wrap_or_flag(desc[4 * c + 3] + q / (CX * CY), BZ, wrap, ok);
    float uv = 0.f, tv = 0.f;
    if (ok) {
        const int pt = boxpt[(z * BY + y) * BX + x];
        if (pt >= 0) {
            const int64_t i = ((int64_t)(k / B) * np + pt) * B + k % B;
            uv = (float)((double)r[i] * inv_s[k]);
            tv = (float)((double)xs[i] * inv_s[k]);
        }
    }
    u[gid] = uv;
    t[gid] = tv;
}

template <typename T> struct OpSumSq {
    const T *x;
    __device__ void operator()(int64_t i, int, double *a) const {
        const double v = x[i];
        a[0] += v * v;
    }
};

// scale: [inv_s | s * g] per state from the sums of squares and shifts.
__global__ void prescale_kernel(const double *__restrict__ ss, const double *__restrict__ sigma,
                                const float *__restrict__ params, double h, int64_t np, int N,
                                double *__restrict__ inv_s, double *__restrict__ outs) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= N) return;
    const double s = sqrt(ss[k] / (double)np);
    const double z = (double)params[kNW] + (double)params[kNW + 1] * log(-sigma[k] * h * h);
    inv_s[k] = s > 0 ? 1.0 / s : 0.0;
    outs[k] = s > 0 ? s * softplus_d(z) : 0.0;
}

__global__ void invs_kernel(const double *__restrict__ ss, int64_t np, int N, double *__restrict__ inv_s) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= N) return;
    const double s = sqrt(ss[k] / (double)np);
    inv_s[k] = s > 0 ? 1.0 / s : 0.0;
}

// ------------------------------------------------- conjugate gradients
template <typename T> struct OpPAp {      // <p|(T - sigma) p> with q = T p
    const T *p, *q;
    const double *sig;
    __device__ void operator()(int64_t i, int c, double *a) const {
        const double pv = p[i];
        a[0] += pv * ((double)q[i] - sig[c] * pv);
    }
};
template <typename T> struct OpCgUpdate { // x += al p, r -= al (q - sigma p), <r|r>
    T *x, *r;
    const T *p, *q;
    const double *sig, *al;
    __device__ void operator()(int64_t i, int c, double *a) const {
        const double pv = p[i], l = al[c];
        x[i] = (T)((double)x[i] + l * pv);
        const double rv = (double)r[i] - l * ((double)q[i] - sig[c] * pv);
        r[i] = (T)rv;
        a[0] += rv * rv;
    }
};

__global__ void cg_alpha_kernel(const double *__restrict__ rr, const double *__restrict__ pap,
                                const int *__restrict__ done, int N, double *__restrict__ al) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= N) return;
    al[k] = (done[k] || !(pap[k] > 0)) ? 0.0 : rr[k] / pap[k];
}

__global__ void cg_beta_kernel(const double *__restrict__ rrn, double *__restrict__ rr,
                               const double *__restrict__ rr0, double tol2, int *__restrict__ done, int N,
                               double *__restrict__ be, int *__restrict__ ndone) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= N) return;
    if (!done[k]) {
        be[k] = rr[k] > 0 ? rrn[k] / rr[k] : 0.0;
        rr[k] = rrn[k];
        if (!(rrn[k] > tol2 * rr0[k])) done[k] = 1;
    } else {
        be[k] = 0.0;
    }
    if (done[k]) atomicAdd(ndone, 1);
}

__global__ void cg_init_kernel(const double *__restrict__ rr, int N, double *__restrict__ rr0,
                               int *__restrict__ done, int *__restrict__ ndone) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k == 0) *ndone = 0;
    if (k >= N) return;
    rr0[k] = rr[k];
    done[k] = rr[k] > 0 ? 0 : 1;
}

__global__ void zero_int_kernel(int *p) { *p = 0; }

template <typename T>
__global__ void __launch_bounds__(256)
cg_p_kernel(T *__restrict__ p, const T *__restrict__ r, const double *__restrict__ be, int64_t np, int B,
            int64_t total) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= total) return;
    const int c = (int)(i / (np * B)) * B + (int)(i % B);
    p[i] = (T)((double)r[i] + be[c] * (double)p[i]);
}

template <typename T>
__global__ void __launch_bounds__(256)
fill_kernel(T *__restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = T(0);
}

}  // namespace

// ================================================================ handle
struct rs_cnn {
    int max_batch = 0;
    int64_t max_box = 0;
    int64_t adam_t = 0;
    rs::DevBuf params, wt, grad, m, v;
    rs::DevBuf a1, a2, f, u;       // forward activations (max_batch * max_box points)
    rs::DevBuf d1, d2, df, t;      // backward deltas (allocated on first training call)
    rs::DevBuf wpart, lpart, gz, coef, loss;
    rs::DevBuf ss, inv_s, outs, partial;   // preconditioner scratch
    // dense box of the last grid used
    const rs_grid *box_grid = nullptr;
    int bdims[3] = {0, 0, 0};      // Z, Y, X
    rs::DevBuf boxpt, boxidx;
};

namespace {

rs_status set_box(rs_cnn *c, const rs_grid *g) {
    if (c->box_grid == g) return RS_OK;
    int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    for (int64_t p = 0; p < g->np; ++p)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], g->inner[3 * p + a]);
            hi[a] = std::max(hi[a], g->inner[3 * p + a]);
        }
    const int X = hi[0] - lo[0] + 1, Y = hi[1] - lo[1] + 1, Z = hi[2] - lo[2] + 1;
    const int64_t vol = (int64_t)X * Y * Z;
    if (vol > c->max_box) return rs::fail(RS_EINVAL, "cnn: the grid's box exceeds max_box of the network handle");
    std::vector<int32_t> pt(vol, -1), idx(g->np);
    for (int64_t p = 0; p < g->np; ++p) {
        const int64_t q = ((int64_t)(g->inner[3 * p + 2] - lo[2]) * Y + (g->inner[3 * p + 1] - lo[1])) * X +
                          (g->inner[3 * p] - lo[0]);
        pt[q] = (int32_t)p;
        idx[p] = (int32_t)q;
    }
    rs_status s = c->boxpt.upload(pt);
    if (!s) s = c->boxidx.upload(idx);
    if (s) return s;
    c->bdims[0] = Z;
    c->bdims[1] = Y;
    c->bdims[2] = X;
    c->box_grid = g;
    return RS_OK;
}

rs_status ensure(rs::DevBuf &b, size_t bytes) { return b.bytes >= bytes ? RS_OK : b.alloc(bytes); }

// f = network(u) for n boxes; activations kept in a1, a2.
rs_status forward(rs_cnn *c, const float *u, float *f, int n, int Z, int Y, int X, int wrap,
                  const int32_t *boxpt, hipStream_t st) {
    const float *P = c->params.as<float>();
    conv<1, 8, 0>(u, c->a1.as<float>(), P + kW1, nullptr, boxpt, n, Z, Y, X, wrap, st);
    {
        const int ntx = (X + kTX - 1) / kTX, nty = (Y + kTY - 1) / kTY, ntz = (Z + kTZ - 1) / kTZ;
        // at most three work-groups per CU resident; each takes tiles in turn
        const int64_t nwg = std::min<int64_t>((int64_t)ntx * nty * ntz * n, 3 * 256);
        hipLaunchKernelGGL(conv2_mfma_kernel, dim3((unsigned)nwg), dim3(256), 0, st, c->a1.as<float>(),
                           c->a2.as<float>(), P + kW2, boxpt, n, Z, Y, X, wrap, ntx, nty, ntz);
    }
    conv<8, 1, 1>(c->a2.as<float>(), f, P + kW3, nullptr, boxpt, n, Z, Y, X, wrap, st);
    RS_HIP(hipGetLastError());
    return RS_OK;
}

rs_status check_batch(rs_cnn *c, int n, const int32_t *dims, const char *who) {
    if (!c || !dims) return rs::fail(RS_EINVAL, std::string(who) + ": null argument");
    if (n < 1 || dims[0] < 1 || dims[1] < 1 || dims[2] < 1) return rs::fail(RS_EINVAL, std::string(who) + ": empty batch");
    const int64_t vol = (int64_t)dims[0] * dims[1] * dims[2];
    if (n > c->max_batch || vol > c->max_box)
        return rs::fail(RS_EINVAL, std::string(who) + ": batch exceeds the handle's max_batch / max_box");
    return RS_OK;
}

}  // namespace

extern "C" rs_status rs_cnn_create(int32_t max_batch, int64_t max_box, rs_cnn **out) {
    using namespace rs;
    if (!out) return fail(RS_EINVAL, "rs_cnn_create: null out");
    *out = nullptr;
    if (max_batch < 1 || max_box < 1 || (int64_t)max_batch * max_box > (int64_t)1 << 28)
        return fail(RS_EINVAL, "rs_cnn_create: need 1 <= max_batch, max_box and max_batch*max_box <= 2^28");
    auto c = new (std::nothrow) rs_cnn();
    if (!c) return fail(RS_ENOMEM, "host allocation failed");
    c->max_batch = max_batch;
    c->max_box = max_box;
    const size_t pts = (size_t)max_batch * max_box;
    rs_status s = c->params.alloc(kNP * sizeof(float));
    if (!s) s = c->wt.alloc(kNW * sizeof(float));
    if (!s) s = c->grad.alloc(kNP * sizeof(float));
    if (!s) s = c->m.alloc(kNP * sizeof(float));
    if (!s) s = c->v.alloc(kNP * sizeof(float));
    if (!s) s = c->a1.alloc(pts * 8 * sizeof(float));
    if (!s) s = c->a2.alloc(pts * 8 * sizeof(float));
    if (!s) s = c->f.alloc(pts * sizeof(float));
    if (!s) s = c->u.alloc(pts * sizeof(float));
    if (!s) s = c->gz.alloc((size_t)std::max(max_batch, 256) * 3 * sizeof(double));
    if (!s) s = c->coef.alloc((size_t)std::max(max_batch, 256) * sizeof(double));
    if (!s) s = c->loss.alloc(sizeof(double));
    if (s) { delete c; return s; }
    std::vector<float> zero(kNP, 0.f);
    if (hipMemcpy(c->params.p, zero.data(), kNP * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->m.p, zero.data(), kNP * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->v.p, zero.data(), kNP * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->grad.p, zero.data(), kNP * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
        delete c;
        return fail(RS_EHIP, "rs_cnn_create: initial copy failed");
    }
    *out = c;
    return RS_OK;
}

extern "C" void rs_cnn_destroy(rs_cnn *c) { delete c; }

extern "C" rs_status rs_cnn_set_params(rs_cnn *c, const float *params) {
    if (!c || !params) return rs::fail(RS_EINVAL, "rs_cnn_set_params: null argument");
    RS_HIP(hipMemcpy(c->params.p, params, kNP * sizeof(float), hipMemcpyHostToDevice));
    std::vector<float> zero(kNP, 0.f);
    RS_HIP(hipMemcpy(c->m.p, zero.data(), kNP * sizeof(float), hipMemcpyHostToDevice));
    RS_HIP(hipMemcpy(c->v.p, zero.data(), kNP * sizeof(float), hipMemcpyHostToDevice));
    c->adam_t = 0;
    return RS_OK;
}

extern "C" rs_status rs_cnn_get_params(const rs_cnn *c, float *params) {
    if (!c || !params) return rs::fail(RS_EINVAL, "rs_cnn_get_params: null argument");
    RS_HIP(hipMemcpy(params, c->params.p, kNP * sizeof(float), hipMemcpyDeviceToHost));
    return RS_OK;
}

// Checkpoint file: 8-byte tag, int64 parameter count, int64 Adam step count,
// then the parameters and the two Adam moments (float each), little endian.
namespace {
constexpr char kCnnTag[8] = {'R', 'S', 'C', 'N', 'N', '0', '0', '1'};
}

extern "C" rs_status rs_cnn_save(const rs_cnn *c, const char *path) {
    using rs::fail;
    if (!c || !path) return fail(RS_EINVAL, "rs_cnn_save: null argument");
    std::vector<float> buf(3 * (size_t)kNP);
    RS_HIP(hipMemcpy(buf.data(), c->params.p, kNP * sizeof(float), hipMemcpyDeviceToHost));
    RS_HIP(hipMemcpy(buf.data() + kNP, c->m.p, kNP * sizeof(float), hipMemcpyDeviceToHost));
    RS_HIP(hipMemcpy(buf.data() + 2 * kNP, c->v.p, kNP * sizeof(float), hipMemcpyDeviceToHost));
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(RS_EINVAL, std::string("rs_cnn_save: cannot open ") + path);
    const int64_t hdr[2] = {(int64_t)kNP, c->adam_t};
    bool ok = std::fwrite(kCnnTag, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(int64_t), 2, f) == 2 &&
              std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return fail(RS_EINVAL, std::string("rs_cnn_save: write failed: ") + path);
    return RS_OK;
}

extern "C" rs_status rs_cnn_load(rs_cnn *c, const char *path) {
    using rs::fail;
    if (!c || !path) return fail(RS_EINVAL, "rs_cnn_load: null argument");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(RS_EINVAL, std::string("rs_cnn_load: cannot open ") + path);
    char tag[8];
    int64_t hdr[2];
    std::vector<float> buf(3 * (size_t)kNP);
    const bool ok = std::fread(tag, 1, 8, f) == 8 && std::memcmp(tag, kCnnTag, 8) == 0 &&
                    std::fread(hdr, sizeof(int64_t), 2, f) == 2 && hdr[0] == kNP && hdr[1] >= 0 &&
                    std::fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    std::fclose(f);
    if (!ok) return fail(RS_EINVAL, std::string("rs_cnn_load: not a network checkpoint of this layout: ") + path);
    RS_HIP(hipMemcpy(c->params.p, buf.data(), kNP * sizeof(float), hipMemcpyHostToDevice));
    RS_HIP(hipMemcpy(c->m.p, buf.data() + kNP, kNP * sizeof(float), hipMemcpyHostToDevice));
    RS_HIP(hipMemcpy(c->v.p, buf.data() + 2 * kNP, kNP * sizeof(float), hipMemcpyHostToDevice));
    c->adam_t = hdr[1];
    return RS_OK;
}

extern "C" rs_status rs_cnn_forward(rs_cnn *c, const float *u, float *f, int32_t n, const int32_t dims[3],
                                    int32_t periodic, void *stream) {
    rs_status s = check_batch(c, n, dims, "rs_cnn_forward");
    if (s) return s;
    if (!u || !f) return rs::fail(RS_EINVAL, "rs_cnn_forward: null field");
    return forward(c, u, f, n, dims[0], dims[1], dims[2], periodic ? 1 : 0, nullptr, (hipStream_t)stream);
}

extern "C" rs_status rs_cnn_loss_grad(rs_cnn *c, const float *u, const float *t, const double *sigma, int32_t n,
                                      const int32_t dims[3], double h, int32_t margin, double *loss, float *grad,
                                      float *du, void *stream) {
    using namespace rs;
    rs_status s = check_batch(c, n, dims, "rs_cnn_loss_grad");
    if (s) return s;
    if (!u || !t || !sigma) return fail(RS_EINVAL, "rs_cnn_loss_grad: null field");
    if (!(h > 0) || margin < 0) return fail(RS_EINVAL, "rs_cnn_loss_grad: bad h or margin");
    hipStream_t st = (hipStream_t)stream;
    const int Z = dims[0], Y = dims[1], X = dims[2];
    const int vol = Z * Y * X;
    const int64_t tot = (int64_t)n * vol;
    const unsigned gsz = (unsigned)((tot + 255) / 256);
    const size_t pts = (size_t)c->max_batch * c->max_box;
    const int nwg = (int)((tot + kWgPts - 1) / kWgPts);
    const int nch = std::max(1, std::min(64, vol / 4096));
    if ((s = ensure(c->d1, pts * 8 * sizeof(float)))) return s;
    if ((s = ensure(c->d2, pts * 8 * sizeof(float)))) return s;
    if ((s = ensure(c->df, pts * sizeof(float)))) return s;
    if ((s = ensure(c->wpart, (size_t)((pts + kWgPts - 1) / kWgPts) * 1728 * sizeof(float)))) return s;
    if ((s = ensure(c->lpart, (size_t)c->max_batch * 64 * 3 * sizeof(double)))) return s;
    const float *P = c->params.as<float>();
    float *G = c->grad.as<float>(), *WT = c->wt.as<float>();
    float *f = c->f.as<float>(), *df = c->df.as<float>();
    float *a1 = c->a1.as<float>(), *a2 = c->a2.as<float>(), *d1 = c->d1.as<float>(), *d2 = c->d2.as<float>();
    if ((s = forward(c, u, f, n, Z, Y, X, 0, nullptr, st))) return s;
    hipLaunchKernelGGL(gain_kernel, dim3((n + 255) / 256), dim3(256), 0, st, P, sigma, h, n, c->gz.as<double>());
    // energy-norm error terms in the (not yet used) delta buffer d1
    float *em = d1, *tm = d1 + tot, *ae = d1 + 2 * tot, *at = d1 + 3 * tot;
    hipLaunchKernelGGL(err_kernel, dim3(gsz), dim3(256), 0, st, f, t, c->gz.as<double>(), Z, Y, X, margin, n, em, tm);
    hipLaunchKernelGGL(kin_kernel, dim3(gsz), dim3(256), 0, st, em, ae, sigma, h, Z, Y, X, n);
    hipLaunchKernelGGL(kin_kernel, dim3(gsz), dim3(256), 0, st, tm, at, sigma, h, Z, Y, X, n);
    hipLaunchKernelGGL(loss_partial_kernel, dim3(nch, n), dim3(256), 0, st, em, ae, tm, at, f, Z, Y, X, margin, nch,
                       c->lpart.as<double>());
    hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(64), 0, st, c->lpart.as<double>(), n, nch,
                       c->gz.as<double>(), c->coef.as<double>(), c->loss.as<double>(), G);
    hipLaunchKernelGGL(df_kernel, dim3(gsz), dim3(256), 0, st, ae, c->gz.as<double>(), c->coef.as<double>(), Z, Y, X,
                       margin, n, df);
    hipLaunchKernelGGL(flip_kernel, dim3((kNW + 255) / 256), dim3(256), 0, st, P, WT);
    RS_HIP(hipGetLastError());
    // layer 3: weights, then delta of layer 2 (through tanh)
    hipLaunchKernelGGL((wgrad_kernel<8, 1>), dim3(nwg), dim3(256), 0, st, a2, df, n, Z, Y, X, 0, c->wpart.as<float>());
    hipLaunchKernelGGL(wgrad_final, dim3((216 + 3) / 4), dim3(256), 0, st, c->wpart.as<float>(), nwg, 216, G + kW3);
    conv<1, 8, 2>(df, d2, WT + kW3, a2, nullptr, n, Z, Y, X, 0, st);
    // layer 2
    hipLaunchKernelGGL((wgrad_kernel<8, 8>), dim3(nwg), dim3(256), 0, st, a1, d2, n, Z, Y, X, 0, c->wpart.as<float>());
    hipLaunchKernelGGL(wgrad_final, dim3((1728 + 3) / 4), dim3(256), 0, st, c->wpart.as<float>(), nwg, 1728, G + kW2);
    conv<8, 8, 2>(d2, d1, WT + kW2, a1, nullptr, n, Z, Y, X, 0, st);
    // layer 1
    hipLaunchKernelGGL((wgrad_kernel<1, 8>), dim3(nwg), dim3(256), 0, st, u, d1, n, Z, Y, X, 0, c->wpart.as<float>());
    hipLaunchKernelGGL(wgrad_final, dim3((216 + 3) / 4), dim3(256), 0, st, c->wpart.as<float>(), nwg, 216, G + kW1);
    if (du)
        conv<8, 1, 1>(d1, du, WT + kW1, nullptr, nullptr, n, Z, Y, X, 0, st);
    RS_HIP(hipGetLastError());
    if (loss) RS_HIP(hipMemcpyAsync(loss, c->loss.p, sizeof(double), hipMemcpyDeviceToHost, st));
    if (grad) RS_HIP(hipMemcpyAsync(grad, G, kNP * sizeof(float), hipMemcpyDeviceToHost, st));
    if (loss || grad) RS_HIP(hipStreamSynchronize(st));
    return RS_OK;
}

extern "C" rs_status rs_cnn_adam_step(rs_cnn *c, float lr, float beta1, float beta2, float eps, void *stream) {
    if (!c) return rs::fail(RS_EINVAL, "rs_cnn_adam_step: null handle");
    if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return rs::fail(RS_EINVAL, "rs_cnn_adam_step: bad hyper-parameters");
    c->adam_t++;
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)c->adam_t));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)c->adam_t));
    hipLaunchKernelGGL(adam_kernel, dim3((kNP + 255) / 256), dim3(256), 0, (hipStream_t)stream, c->params.as<float>(),
                       c->grad.as<float>(), c->m.as<float>(), c->v.as<float>(), lr, beta1, beta2, eps, c1, c2);
    RS_HIP(hipGetLastError());
    return RS_OK;
}

namespace rs {

// out = K(r) for nblk blocks of B states; sigma DEVICE double [nblk*B].
rs_status cnn_precondition(rs_cnn *c, const rs_grid *g, const void *r, const double *sigma, void *out, int nblk,
                           int B, int dtype, hipStream_t st) {
    rs_status s = set_box(c, g);
    if (s) return s;
    const int Z = c->bdims[0], Y = c->bdims[1], X = c->bdims[2];
    const int vol = Z * Y * X;
    const int N = nblk * B;
    const int cb = c->max_batch / B;          // blocks per chunk
    if (cb < 1) return fail(RS_EINVAL, "cnn precondition: max_batch of the network handle is below B");
    const int64_t np = g->np;
    const int nchunks = (int)((np + kChunk - 1) / kChunk);
    if ((s = ensure(c->ss, (size_t)N * sizeof(double)))) return s;
    if ((s = ensure(c->inv_s, (size_t)N * sizeof(double)))) return s;
    if ((s = ensure(c->outs, (size_t)N * sizeof(double)))) return s;
    if ((s = ensure(c->partial, (size_t)nchunks * N * sizeof(double)))) return s;
    if (dtype == RS_F64)
        s = colreduce<1>(OpSumSq<double>{(const double *)r}, np, B, nblk, 1.0, c->partial.as<double>(),
                         c->ss.as<double>(), st);
    else
        s = colreduce<1>(OpSumSq<float>{(const float *)r}, np, B, nblk, 1.0, c->partial.as<double>(),
                         c->ss.as<double>(), st);
    if (s) return s;
    hipLaunchKernelGGL(prescale_kernel, dim3((N + 255) / 256), dim3(256), 0, st, c->ss.as<double>(), sigma,
                       c->params.as<float>(), g->h, np, N, c->inv_s.as<double>(), c->outs.as<double>());
    const int wrap = g->kind == RS_GRID_PERIODIC ? 1 : 0;
    for (int b0 = 0; b0 < nblk; b0 += cb) {
        const int nb = std::min(cb, nblk - b0);
        const int k0 = b0 * B;
        if (dtype == RS_F64)
            hipLaunchKernelGGL(scatter_kernel<double>, dim3((vol + 63) / 64, nb), dim3(256), 0, st, (const double *)r,
                               c->boxpt.as<int32_t>(), c->inv_s.as<double>(), k0, B, np, vol, c->u.as<float>());
        else
            hipLaunchKernelGGL(scatter_kernel<float>, dim3((vol + 63) / 64, nb), dim3(256), 0, st, (const float *)r,
                               c->boxpt.as<int32_t>(), c->inv_s.as<double>(), k0, B, np, vol, c->u.as<float>());
        RS_HIP(hipGetLastError());
        if ((s = forward(c, c->u.as<float>(), c->f.as<float>(), nb * B, Z, Y, X, wrap, c->boxpt.as<int32_t>(), st)))
            return s;
        if (dtype == RS_F64)
            hipLaunchKernelGGL(gather_kernel<double>, dim3((unsigned)((np + 63) / 64), nb), dim3(256), 0, st,
                               c->f.as<float>(), c->boxidx.as<int32_t>(), c->outs.as<double>(), k0, B, np, vol,
                               (double *)out);
        else
            hipLaunchKernelGGL(gather_kernel<float>, dim3((unsigned)((np + 63) / 64), nb), dim3(256), 0, st,
                               c->f.as<float>(), c->boxidx.as<int32_t>(), c->outs.as<double>(), k0, B, np, vol,
                               (float *)out);
        RS_HIP(hipGetLastError());
    }
    return RS_OK;
}

rs_status check_fields_cnn(const rs_grid *g, int nblk, int B, int dtype, const char *who) {
    if (!g) return fail(RS_EINVAL, std::string(who) + ": null grid");
    if (g->host_only) return fail(RS_EINVAL, std::string(who) + ": grid was built host-only");
    if (!g->kernels_ok) return fail(RS_ENOTSUP, std::string(who) + ": kernels need 4x4x4 bricks");
    if (B < 1 || B > 64 || (B & (B - 1))) return fail(RS_EINVAL, std::string(who) + ": B must be a power of two <= 64");
    if (nblk < 1 || nblk > 65535) return fail(RS_EINVAL, std::string(who) + ": bad nblk");
    if (dtype != RS_F64 && dtype != RS_F32) return fail(RS_EINVAL, std::string(who) + ": bad dtype");
    return RS_OK;
}

}  // namespace rs

extern "C" rs_status rs_cnn_precondition(rs_cnn *c, const rs_grid *g, const void *r, const double *sigma, void *out,
                                         int32_t nblk, int32_t B, int32_t dtype, void *stream) {
    using namespace rs;
    if (!c || !r || !sigma || !out) return fail(RS_EINVAL, "rs_cnn_precondition: null argument");
    rs_status s = check_fields_cnn(g, nblk, B, dtype, "rs_cnn_precondition");
    if (s) return s;
    if (r == out) return fail(RS_EINVAL, "rs_cnn_precondition: r and out must differ");
    return cnn_precondition(c, g, r, sigma, out, nblk, B, dtype, (hipStream_t)stream);
}

extern "C" rs_status rs_cnn_crops(rs_cnn *c, const rs_grid *g, const void *r, const void *x, int32_t nblk, int32_t B,
                                  int32_t dtype, int32_t ncrops, const int32_t *desc, const int32_t cdims[3],
                                  float *u_out, float *t_out, void *stream) {
    using namespace rs;
    if (!c || !r || !x || !desc || !cdims || !u_out || !t_out) return fail(RS_EINVAL, "rs_cnn_crops: null argument");
    rs_status s = check_fields_cnn(g, nblk, B, dtype, "rs_cnn_crops");
    if (s) return s;
    if (ncrops < 1 || cdims[0] < 1 || cdims[1] < 1 || cdims[2] < 1)
        return fail(RS_EINVAL, "rs_cnn_crops: empty crop set");
    if ((int64_t)ncrops * cdims[0] * cdims[1] * cdims[2] > ((int64_t)1 << 31) - 1)
        return fail(RS_EINVAL, "rs_cnn_crops: too many crop points");
    if ((s = set_box(c, g))) return s;
    const int N = nblk * B;
    const int BZ = c->bdims[0], BY = c->bdims[1], BX = c->bdims[2];
    for (int i = 0; i < ncrops; ++i) {
        const int32_t *d = desc + 4 * i;
        if (d[0] < 0 || d[0] >= N || d[1] < 0 || d[1] >= BX || d[2] < 0 || d[2] >= BY || d[3] < 0 || d[3] >= BZ)
            return fail(RS_EINVAL, "rs_cnn_crops: crop state or origin out of range");
    }
    hipStream_t st = (hipStream_t)stream;
    const int64_t np = g->np;
    const int nchunks = (int)((np + kChunk - 1) / kChunk);
    if ((s = ensure(c->ss, (size_t)N * sizeof(double)))) return s;
    if ((s = ensure(c->inv_s, (size_t)N * sizeof(double)))) return s;
    if ((s = ensure(c->partial, (size_t)nchunks * N * sizeof(double)))) return s;
    rs::DevBuf ddesc;
    if ((s = ddesc.upload(std::vector<int32_t>(desc, desc + 4 * (size_t)ncrops)))) return s;
    if (dtype == RS_F64)
        s = colreduce<1>(OpSumSq<double>{(const double *)r}, np, B, nblk, 1.0, c->partial.as<double>(),
                         c->ss.as<double>(), st);
    else
        s = colreduce<1>(OpSumSq<float>{(const float *)r}, np, B, nblk, 1.0, c->partial.as<double>(),
                         c->ss.as<double>(), st);
    if (s) return s;
    hipLaunchKernelGGL(invs_kernel, dim3((N + 255) / 256), dim3(256), 0, st, c->ss.as<double>(), np, N,
                       c->inv_s.as<double>());
    const int wrap = g->kind == RS_GRID_PERIODIC ? 1 : 0;
    const int64_t tot = (int64_t)ncrops * cdims[0] * cdims[1] * cdims[2];
    const unsigned gsz = (unsigned)((tot + 255) / 256);
    if (dtype == RS_F64)
        hipLaunchKernelGGL(crop_kernel<double>, dim3(gsz), dim3(256), 0, st, (const double *)r, (const double *)x,
                           c->boxpt.as<int32_t>(), ddesc.as<int32_t>(), c->inv_s.as<double>(), B, np, BZ, BY, BX, wrap,
                           cdims[0], cdims[1], cdims[2], ncrops, u_out, t_out);
    else
        hipLaunchKernelGGL(crop_kernel<float>, dim3(gsz), dim3(256), 0, st, (const float *)r, (const float *)x,
                           c->boxpt.as<int32_t>(), ddesc.as<int32_t>(), c->inv_s.as<double>(), B, np, BZ, BY, BX, wrap,
                           cdims[0], cdims[1], cdims[2], ncrops, u_out, t_out);
    RS_HIP(hipGetLastError());
    RS_HIP(hipStreamSynchronize(st));   // the descriptor buffer is freed on return
    return RS_OK;
}

extern "C" rs_status rs_cnn_box(rs_cnn *c, const rs_grid *g, int32_t dims[3]) {
    if (!c || !g || !dims) return rs::fail(RS_EINVAL, "rs_cnn_box: null argument");
    rs_status s = set_box(c, g);
    if (s) return s;
    for (int a = 0; a < 3; ++a) dims[a] = c->bdims[a];
    return RS_OK;
}

// ------------------------------------------------------ shifted solves
namespace {

template <typename T>
rs_status shifted_cg(const rs_grid *g, const T *b, const double *sigma, T *x, int nblk, int B, double tol, int maxit,
                     int *iters, hipStream_t st) {
    using namespace rs;
    const int N = nblk * B;
    const int64_t np = g->np, total = np * N;
    const size_t bytes = (size_t)total * sizeof(T);
    const int nchunks = (int)((np + kChunk - 1) / kChunk);
    rs::DevBuf r, p, q, partial, small, flags;
    rs_status s = r.alloc(bytes);
    if (!s) s = p.alloc(bytes);
    if (!s) s = q.alloc(bytes);
    if (!s) s = partial.alloc((size_t)nchunks * N * sizeof(double));
    if (!s) s = small.alloc((size_t)6 * N * sizeof(double));
    if (!s) s = flags.alloc((size_t)(N + 1) * sizeof(int));
    if (s) return s;
    double *rr = small.as<double>(), *rr0 = rr + N, *pap = rr + 2 * N, *rrn = rr + 3 * N, *al = rr + 4 * N,
           *be = rr + 5 * N;
    int *done = flags.as<int>(), *ndone = done + N;
    const unsigned gm = (unsigned)((total + 255) / 256), gs = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(fill_kernel<T>, dim3(gm), dim3(256), 0, st, x, total);
    RS_HIP(hipMemcpyAsync(r.p, b, bytes, hipMemcpyDeviceToDevice, st));
    RS_HIP(hipMemcpyAsync(p.p, b, bytes, hipMemcpyDeviceToDevice, st));
    if ((s = colreduce<1>(OpSumSq<T>{b}, np, B, nblk, 1.0, partial.as<double>(), rr, st))) return s;
    hipLaunchKernelGGL(cg_init_kernel, dim3(gs), dim3(256), 0, st, rr, N, rr0, done, ndone);
    RS_HIP(hipGetLastError());
    const double tol2 = tol * tol;
    int it = 0;
    int nd = 0;
    while (it < maxit) {
        if ((s = kinetic_apply(g, p.p, q.p, nblk, B, sizeof(T) == 8 ? RS_F64 : RS_F32, st))) return s;
        if ((s = colreduce<1>(OpPAp<T>{p.as<T>(), q.as<T>(), sigma}, np, B, nblk, 1.0, partial.as<double>(), pap, st)))
            return s;
        hipLaunchKernelGGL(cg_alpha_kernel, dim3(gs), dim3(256), 0, st, rr, pap, done, N, al);
        if ((s = colreduce<1>(OpCgUpdate<T>{x, r.as<T>(), p.as<T>(), q.as<T>(), sigma, al}, np, B, nblk, 1.0,
                              partial.as<double>(), rrn, st)))
            return s;
        hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, st, ndone);
        hipLaunchKernelGGL(cg_beta_kernel, dim3(gs), dim3(256), 0, st, rrn, rr, rr0, tol2, done, N, be, ndone);
        hipLaunchKernelGGL(cg_p_kernel<T>, dim3(gm), dim3(256), 0, st, p.as<T>(), r.as<T>(), be, np, B, total);
        RS_HIP(hipGetLastError());
        ++it;
        if (it % 10 == 0 || it == maxit) {
            RS_HIP(hipMemcpyAsync(&nd, ndone, sizeof(int), hipMemcpyDeviceToHost, st));
            RS_HIP(hipStreamSynchronize(st));
            if (nd == N) break;
        }
    }
    RS_HIP(hipStreamSynchronize(st));   // scratch is freed on return
    if (iters) *iters = it;
    return nd == N ? RS_OK : fail(RS_ENOTCONV, "rs_shifted_solve: not converged within maxit");
}

}  // namespace

extern "C" rs_status rs_shifted_solve(const rs_grid *g, const void *r, const double *sigma, void *x, int32_t nblk,
                                      int32_t B, int32_t dtype, double tol, int32_t maxit, int32_t *iters,
                                      void *stream) {
    using namespace rs;
    rs_status s = check_fields_cnn(g, nblk, B, dtype, "rs_shifted_solve");
    if (s) return s;
    if (!r || !sigma || !x || r == x) return fail(RS_EINVAL, "rs_shifted_solve: null or aliased argument");
    if (!(tol > 0) || maxit < 1) return fail(RS_EINVAL, "rs_shifted_solve: bad tol or maxit");
    hipStream_t st = (hipStream_t)stream;
    if (dtype == RS_F64)
        return shifted_cg<double>(g, (const double *)r, sigma, (double *)x, nblk, B, tol, maxit, iters, st);
    return shifted_cg<float>(g, (const float *)r, sigma, (float *)x, nblk, B, tol, maxit, iters, st);
}
