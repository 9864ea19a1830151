// Hartree potential by FFT on an enlarged cubic box (Sec. 7, eq. (5)).
//
// The density on the domain's points is placed in an N^3 box (zeros
// elsewhere), transformed by a 3-D complex FFT, multiplied by the Coulomb
// interaction cut off at R_c,
//     v(k) = 4 pi / k^2 (1 - cos(k R_c)),  v(0) = 2 pi R_c^2,
// transformed back and read out at the domain's points.  R_c bounds every
// pair distance in the domain and the box is longer than the domain's span
// plus R_c on every axis, so no periodic image of the density comes within
// R_c of a domain point: on the domain the result is the free-space
// potential int n(r') / |r - r'| d^3r'.
//
// The FFT is three passes of 1-D transforms along x, y and z.  A work-group
// loads LB lines into LDS (lines chosen so that the loads are contiguous in
// memory: whole x lines, or LB neighbouring lines for y and z), runs a
// radix-2 decimation-in-time transform in place (bit-reversed load, log2 N
// butterfly stages with one barrier each) and writes the lines back.
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace {

typedef double2 cplx;

constexpr int kPoissonMinN = 16, kPoissonMaxN = 512;

__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
    return cplx{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

__device__ __forceinline__ int bitrev(int j, int logn) { return (int)(__brev((unsigned)j) >> (32 - logn)); }

// One pass of 1-D transforms of length N.  Line (g, i), g the work-group,
// i in [0, LB): base = (g / G2) S1 + (g % G2) S2 + i S_line; element j at
// base + j S_elem.  CONTIG: S_elem == 1 (lines are contiguous; j runs
// fastest over the threads), else S_line == 1 (neighbouring lines are
// contiguous; i runs fastest).  tw[k] = exp(-2 pi i k / N), k < N/2;
// inverse transforms use the conjugates.
template <int N, int LB, bool CONTIG>
__global__ void __launch_bounds__(256)
fft_pass_kernel(cplx *__restrict__ data, int64_t S_elem, int64_t S_line, int64_t S1, int64_t S2, int G2,
                const cplx *__restrict__ tw, int inverse) {
    constexpr int LOGN = __builtin_ctz(N);
    __shared__ cplx buf[LB * N];
    const int g = blockIdx.x;
    const int64_t base = (int64_t)(g / G2) * S1 + (int64_t)(g % G2) * S2;
    const int tid = threadIdx.x;
    for (int e = tid; e < LB * N; e += 256) {
        const int i = CONTIG ? e / N : e % LB;
        const int j = CONTIG ? e % N : e / LB;
        buf[i * N + bitrev(j, LOGN)] = data[base + i * S_line + j * S_elem];
    }
    __syncthreads();
    for (int s = 0; s < LOGN; ++s) {
        const int half = 1 << s;
        for (int b = tid; b < LB * (N / 2); b += 256) {
            const int i = b / (N / 2), t = b % (N / 2);
            const int grp = t >> s, pos = t & (half - 1);
            const int i0 = i * N + grp * 2 * half + pos, i1 = i0 + half;
            cplx w = tw[pos << (LOGN - 1 - s)];
            if (inverse) w.y = -w.y;
            const cplx u = buf[i0], v = cmul(w, buf[i1]);
            buf[i0] = cplx{u.x + v.x, u.y + v.y};
            buf[i1] = cplx{u.x - v.x, u.y - v.y};
        }
        __syncthreads();
    }
    for (int e = tid; e < LB * N; e += 256) {
        const int i = CONTIG ? e / N : e % LB;
        const int j = CONTIG ? e % N : e / LB;
        data[base + i * S_line + j * S_elem] = buf[i * N + j];
    }
}

__global__ void __launch_bounds__(256) box_zero_kernel(cplx *__restrict__ box, int64_t n3) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < n3) box[e] = cplx{0.0, 0.0};
}

__global__ void __launch_bounds__(256)
scatter_kernel(const double *__restrict__ rho, const int64_t *__restrict__ pts, int64_t np, cplx *__restrict__ box) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < np) box[pts[p]] = cplx{rho[p], 0.0};
}

__global__ void __launch_bounds__(256)
gather_kernel(const cplx *__restrict__ box, const int64_t *__restrict__ pts, int64_t np, double *__restrict__ v) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < np) v[p] = box[pts[p]].x;
}

// box *= v(k) / N^3, k = 2 pi m / (N h) with m the signed DFT frequency.
__global__ void __launch_bounds__(256)
kernel_multiply(cplx *__restrict__ box, int n, double dk, double rc, double scale) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n3 = (int64_t)n * n * n;
    if (e >= n3) return;
    const int x = (int)(e % n), y = (int)((e / n) % n), z = (int)(e / ((int64_t)n * n));
    const double kx = (x < n / 2 ? x : x - n) * dk, ky = (y < n / 2 ? y : y - n) * dk,
                 kz = (z < n / 2 ? z : z - n) * dk;
    const double k2 = (kx * kx + ky * ky) + kz * kz;
    double vk;
    if (k2 > 0.0) {
        const double k = sqrt(k2);
        vk = 4.0 * M_PI / k2 * (1.0 - cos(k * rc));
    } else {
        vk = 2.0 * M_PI * rc * rc;
    }
    const double f = vk * scale;
    box[e] = cplx{box[e].x * f, box[e].y * f};
}

}  // namespace

struct rs_poisson {
    const rs_grid *g = nullptr;
    int n = 0;
    double rc = 0.0;
    rs::DevBuf box;    // complex double [n^3]
    rs::DevBuf pts;    // int64 [np]: box index of each inner point
    rs::DevBuf tw;     // complex double [n/2]
};

namespace {

template <int N>
rs_status fft3d(cplx *box, const cplx *tw, int inverse, hipStream_t st) {
    constexpr int LBX = 4, LBYZ = N >= 512 ? 4 : 8;
    const int64_t n = N, n2 = n * n;
    // x: lines (z, y), 4 neighbouring y per group; contiguous elements
    hipLaunchKernelGGL((fft_pass_kernel<N, LBX, true>), dim3((unsigned)(n2 / LBX)), dim3(256), 0, st, box, (int64_t)1,
                       n, n2, LBX * n, (int)(N / LBX), tw, inverse);
    RS_HIP(hipGetLastError());
    // y: lines (z, x), LBYZ neighbouring x per group
    hipLaunchKernelGGL((fft_pass_kernel<N, LBYZ, false>), dim3((unsigned)(n2 / LBYZ)), dim3(256), 0, st, box, n,
                       (int64_t)1, n2, (int64_t)LBYZ, (int)(N / LBYZ), tw, inverse);
    RS_HIP(hipGetLastError());
    // z: lines (y, x)
    hipLaunchKernelGGL((fft_pass_kernel<N, LBYZ, false>), dim3((unsigned)(n2 / LBYZ)), dim3(256), 0, st, box, n2,
                       (int64_t)1, n, (int64_t)LBYZ, (int)(N / LBYZ), tw, inverse);
    RS_HIP(hipGetLastError());
    return RS_OK;
}

rs_status fft3d_any(int n, cplx *box, const cplx *tw, int inverse, hipStream_t st) {
    switch (n) {
        case 16: return fft3d<16>(box, tw, inverse, st);
        case 32: return fft3d<32>(box, tw, inverse, st);
        case 64: return fft3d<64>(box, tw, inverse, st);
        case 128: return fft3d<128>(box, tw, inverse, st);
        case 256: return fft3d<256>(box, tw, inverse, st);
        case 512: return fft3d<512>(box, tw, inverse, st);
    }
    return rs::fail(RS_ENOTSUP, "poisson: FFT box edge must be a power of two in [16, 512]");
}

}  // namespace

extern "C" rs_status rs_poisson_create(const rs_grid *g, rs_poisson **out) {
    using rs::fail;
    if (!g || !out) return fail(RS_EINVAL, "rs_poisson_create: null argument");
    *out = nullptr;
    if (g->host_only) return fail(RS_EINVAL, "rs_poisson_create: host-only grid");
    if (g->kind == RS_GRID_PERIODIC) return fail(RS_EINVAL, "rs_poisson_create: the free-boundary solve is for finite systems");
    if (g->np < 1) return fail(RS_EINVAL, "rs_poisson_create: empty grid");
    int32_t lo[3], hi[3];
    for (int a = 0; a < 3; ++a) { lo[a] = g->inner[a]; hi[a] = g->inner[a]; }
    for (int64_t p = 1; p < g->np; ++p)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], g->inner[3 * p + a]);
            hi[a] = std::max(hi[a], g->inner[3 * p + a]);
        }
    // R_c: twice the largest distance from the bounding box's centre
    double m = 0.0;
    for (int64_t p = 0; p < g->np; ++p) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double d = (double)g->inner[3 * p + a] - 0.5 * ((double)lo[a] + (double)hi[a]);
            s += d * d;
        }
        m = std::max(m, s);
    }
    const double rc = (2.0 * g->h) * std::sqrt(m);
    int ext = 0;
    for (int a = 0; a < 3; ++a) ext = std::max(ext, hi[a] - lo[a] + 1);
    int n = 2;
    while (!((double)n > (double)(ext - 1) + rc / g->h)) n *= 2;
    if (n < kPoissonMinN) n = kPoissonMinN;
    if (n > kPoissonMaxN) return fail(RS_ENOTSUP, "rs_poisson_create: the domain needs an FFT box above 512^3");
    auto p = new (std::nothrow) rs_poisson();
    if (!p) return fail(RS_ENOMEM, "host allocation failed");
    p->g = g;
    p->n = n;
    p->rc = rc;
    std::vector<int64_t> idx(g->np);
    for (int64_t q = 0; q < g->np; ++q) {
        const int64_t x = g->inner[3 * q] - lo[0], y = g->inner[3 * q + 1] - lo[1], z = g->inner[3 * q + 2] - lo[2];
        idx[q] = (z * n + y) * n + x;
    }
    std::vector<cplx> tw(n / 2);
    for (int k = 0; k < n / 2; ++k) {
        const double a = -2.0 * M_PI * (double)k / (double)n;
        tw[k] = cplx{std::cos(a), std::sin(a)};
    }
    rs_status s = p->box.alloc((size_t)n * n * n * sizeof(cplx));
    if (!s) s = p->pts.alloc(sizeof(int64_t) * g->np);
    if (!s) s = p->tw.alloc(sizeof(cplx) * (n / 2));
    if (s) { delete p; return s; }
    hipError_t e = hipMemcpy(p->pts.p, idx.data(), sizeof(int64_t) * g->np, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->tw.p, tw.data(), sizeof(cplx) * (n / 2), hipMemcpyHostToDevice);
    if (e != hipSuccess) { delete p; return rs::hip_fail(e, "rs_poisson_create: upload"); }
    *out = p;
    return RS_OK;
}

extern "C" void rs_poisson_destroy(rs_poisson *p) { delete p; }

extern "C" rs_status rs_poisson_info(const rs_poisson *p, int32_t *nbox, double *rc) {
    if (!p) return rs::fail(RS_EINVAL, "rs_poisson_info: null handle");
    if (nbox) *nbox = p->n;
    if (rc) *rc = p->rc;
    return RS_OK;
}

extern "C" rs_status rs_poisson_solve(rs_poisson *p, const double *rho, double *vh, void *stream) {
    using namespace rs;
    if (!p || !rho || !vh) return fail(RS_EINVAL, "rs_poisson_solve: null argument");
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = p->n, n3 = n * n * n, np = p->g->np;
    cplx *box = p->box.as<cplx>();
    const cplx *tw = p->tw.as<cplx>();
    hipLaunchKernelGGL(box_zero_kernel, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, st, box, n3);
    RS_HIP(hipGetLastError());
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, rho,
                       p->pts.as<int64_t>(), np, box);
    RS_HIP(hipGetLastError());
    rs_status s = fft3d_any(p->n, box, tw, 0, st);
    if (s) return s;
    const double dk = 2.0 * M_PI * (1.0 / ((double)n * p->g->h));
    hipLaunchKernelGGL(kernel_multiply, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, st, box, p->n, dk, p->rc,
                       1.0 / (double)n3);
    RS_HIP(hipGetLastError());
    if ((s = fft3d_any(p->n, box, tw, 1, st))) return s;
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, box, p->pts.as<int64_t>(),
                       np, vh);
    RS_HIP(hipGetLastError());
    return RS_OK;
}
