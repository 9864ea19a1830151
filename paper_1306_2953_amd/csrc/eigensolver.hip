// One RMM-DIIS eigensolver step on gfx950 (Secs. 3, 6 and 9).
//
// The step, for N states in nblk blocks of B (all on the caller's stream,
// one host synchronisation at the end):
//   1. H psi for all blocks; Rayleigh-Ritz (subspace matrix, Jacobi, rotate).
//   2. Per state: eps0 = <psi|H psi>/<psi|psi>, R0 = H psi - eps0 psi,
//      residual norm.  A block whose states are all below tol is frozen.
//   3. d = K R0 (filter), H d; the trial step lambda minimises the Rayleigh
//      quotient of psi + lambda d (2x2 generalised problem per state);
//      psi1 = psi + lambda d, H psi1 = H psi + lambda H d.  With a learned
//      preconditioner its direction d_n = K_n R0 joins the filter's: the
//      Rayleigh quotient is minimised over span{psi, d_f, d_n} (3x3 problem
//      per state), giving K = a K_f + b K_n for the state's step (lambda 1);
//      a singular 3x3 problem leaves the state on the filter (b = 0).
//   4. m - 1 DIIS iterations: residuals R_i = H psi_i - eps_i psi_i of the
//      history; minimise |sum c R| / |sum c psi| over the history written in
//      the basis {psi_L, psi_i - psi_L} (generalised eigenproblem per state,
//      lowest eigenvector, c_0 = 1); psi_bar, H psi_bar, R_bar; d = K R_bar;
//      psi_{j+1} = psi_bar + lambda d, H psi_{j+1} = H psi_bar + lambda H d.
//   5. Orthonormalise (Cholesky, eq. 8).
// Per-state inner products are sums over points with FP64 accumulation and
// a fixed-order reduction over point chunks; the small per-state problems
// are solved in FP64, one thread per state.
#include <cmath>
#include <cstring>

#include "colreduce.hpp"
#include "dense.hpp"
#include "internal.hpp"

rs_status subspace_diag_capped(rs_ctx *c, void *psi, void *hpsi, double *eig, int nblk, int B, int dtype,
                               int prec, int max_sweeps, int nreal, hipStream_t st);
rs_status orthonormalize_impl(rs_ctx *c, void *psi, int nblk, int B, int dtype, int prec, double *S_out,
                              int32_t *info, int nreal, hipStream_t s);
const int *ctx_sweeps(const rs_ctx *c);

namespace rs {
rs_status hpsi_apply(const rs_grid *g, const rs_nl *nl, const void *vloc, const void *psi, void *hpsi,
                     int nblk, int B, int dtype, hipStream_t st);
rs_status filter_apply(const rs_grid *g, double alpha, const void *r, void *out, int nblk, int B, int dtype,
                       hipStream_t st);
rs_status kinetic_apply(const rs_grid *g, const void *psi, void *out, int nblk, int B, int dtype,
                        hipStream_t st);
rs_status cnn_precondition(rs_cnn *c, const rs_grid *g, const void *r, const double *sigma, void *out, int nblk,
                           int B, int dtype, hipStream_t st);
}

namespace {
using namespace rsred;

constexpr int kMaxHist = 4;   // iterates kept (m <= 3)
constexpr int kMaxSweeps = 30;  // Jacobi sweeps that reach FP64 accuracy from any start

template <typename T> struct OpDots2 {   // <x|x>, <x|y>
    const T *x, *y;
    __device__ void operator()(int64_t i, int, double *a) const {
        const double u = x[i], v = y[i];
        a[0] += u * u;
        a[1] += u * v;
    }
};
// y = x + lambda d, hy = hx + lambda hd (per-state lambda; in place when
// y == x), and the dots <y|y>, <y|hy> of the new iterate for its Rayleigh
// quotient.
template <typename T> struct OpAxpy2Dots {
    const T *x, *hx, *d, *hd;
    T *y, *hy;
    const double *lam;
    __device__ void operator()(int64_t i, int c, double *a) const {
        const double l = lam[c];
        const T yv = (T)((double)x[i] + l * (double)d[i]);
        const T hv = (T)((double)hx[i] + l * (double)hd[i]);
        y[i] = yv;
        hy[i] = hv;
        a[0] += (double)yv * (double)yv;
        a[1] += (double)yv * (double)hv;
    }
};
// The first DIIS pass over iterates 0 and 1 with iterate 1 formed on the
// fly: y = x + lambda d, hy = hx + lambda hd (stored, rounded to T, for the
// later passes), and the DIIS matrices of {x, y} as OpDiis<T, 2> forms them
// from the stored values.  eps[N + c] (iterate 1's Rayleigh quotient) comes
// from the trial-step dots, so no separate pass writes iterate 1.
template <typename T> struct OpDiis2New {
    const T *x, *hx, *d, *hd;
    T *y, *hy;
    const double *lam, *eps;
    int N;
    __device__ void operator()(int64_t i, int c, double *a) const {
        const double l = lam[c];
        const double u = x[i], hu = hx[i];
        const T yv = (T)(u + l * (double)d[i]);
        const T hv = (T)(hu + l * (double)hd[i]);
        y[i] = yv;
        hy[i] = hv;
        const double xl = yv, rl = (double)hv - eps[N + c] * xl;
        const double e1 = u - xl, r1 = (hu - eps[c] * u) - rl;
        a[0] += rl * rl;
        a[1] += rl * r1;
        a[2] += r1 * r1;
        a[3] += xl * xl;
        a[4] += xl * e1;
        a[5] += e1 * e1;
    }
};
template <typename T> struct OpResid {   // R = h - eps x, <R|R>
    const T *x, *h;
    T *R;
    const double *eps;
    __device__ void operator()(int64_t i, int c, double *a) const {
        const T r = (T)((double)h[i] - eps[c] * (double)x[i]);
        R[i] = r;
        a[0] += (double)r * (double)r;
    }
};
template <typename T> struct OpLam {     // <x|Hd>, <d|Hx>, <d|Hd>, <x|d>, <d|d>
    const T *x, *hx, *d, *hd;
    __device__ void operator()(int64_t i, int, double *a) const {
        const double u = x[i], hu = hx[i], v = d[i], hv = hd[i];
        a[0] += u * hv;
        a[1] += v * hu;
        a[2] += v * hv;
        a[3] += u * v;
        a[4] += v * v;
    }
};
// The trial subspace {x, d, e} (filter and network directions): <x|Hd>,
// <d|Hx>, <d|Hd>, <x|d>, <d|d>, the same five for e, then <d|He>, <e|Hd>,
// <d|e>.
template <typename T> struct OpLam3 {
    const T *x, *hx, *d, *hd, *e, *he;
    __device__ void operator()(int64_t i, int, double *a) const {
        const double u = x[i], hu = hx[i], v = d[i], hv = hd[i], w = e[i], hw = he[i];
        a[0] += u * hv;
        a[1] += v * hu;
        a[2] += v * hv;
        a[3] += u * v;
        a[4] += v * v;
        a[5] += u * hw;
        a[6] += w * hu;
        a[7] += w * hw;
        a[8] += u * w;
        a[9] += w * w;
        a[10] += v * hw;
        a[11] += w * hv;
        a[12] += v * w;
    }
};
// DIIS matrices over n = L + 1 iterates in the basis {x_L, x_i - x_L}:
// A_ab = <r_a|r_b>, B_ab = <e_a|e_b> (upper triangles, 2 * n(n+1)/2 values)
template <typename T, int NIT> struct OpDiis {
    const T *x[NIT], *h[NIT];
    const double *eps;   // [NIT][N]
    int N;
    __device__ void operator()(int64_t i, int c, double *a) const {
        double e[NIT], r[NIT];
        const double xl = x[NIT - 1][i];
        const double rl = (double)h[NIT - 1][i] - eps[(NIT - 1) * N + c] * xl;
        e[0] = xl;
        r[0] = rl;
#pragma unroll
        for (int k = 0; k < NIT - 1; ++k) {
            const double xk = x[k][i];
            e[k + 1] = xk - xl;
            r[k + 1] = ((double)h[k][i] - eps[k * N + c] * xk) - rl;
        }
        int t = 0;
#pragma unroll
        for (int p = 0; p < NIT; ++p)
#pragma unroll
            for (int q = p; q < NIT; ++q) {
                a[t] += r[p] * r[q];
                a[t + NIT * (NIT + 1) / 2] += e[p] * e[q];
                ++t;
            }
    }
};

// --------------------------------------------------------- map kernels
// y = x + lambda d (the newest iterate, written straight into psi)
template <typename T>
__global__ void __launch_bounds__(256)
axpy1_kernel(const T *__restrict__ x, const T *__restrict__ d, T *y, const double *__restrict__ lam, int64_t np,
             int B, const int *__restrict__ bmap) {
    // blockIdx.y: the block (or its entry in the block map); B is a power of two
    const int blk = bmap ? bmap[blockIdx.y] : (int)blockIdx.y;
    const int64_t il = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (il >= np * B) return;
    const int64_t i = (int64_t)blk * np * B + il;
    const int c = blk * B + (int)(il & (B - 1));
    y[i] = (T)((double)x[i] + lam[c] * (double)d[i]);
}

// psi_bar = sum_a c_a e_a, H psi_bar = sum_a c_a he_a (skipped when hb is
// null), R_bar = sum_a c_a r_a
template <typename T> struct Hist {
    const T *x[kMaxHist], *h[kMaxHist];
};

template <typename T, int NIT>
__global__ void __launch_bounds__(256)
combine_kernel(Hist<T> H, const double *__restrict__ eps, const double *__restrict__ coef, T *__restrict__ xb,
               T *__restrict__ hb, T *__restrict__ rb, int64_t np, int B, int N, const int *__restrict__ bmap) {
    const T *const *xs = H.x;
    const T *const *hs = H.h;
    // blockIdx.y: the block (or its entry in the block map); B is a power of two
    const int blk = bmap ? bmap[blockIdx.y] : (int)blockIdx.y;
    const int64_t il = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (il >= np * B) return;
    const int64_t i = (int64_t)blk * np * B + il;
    const int c = blk * B + (int)(il & (B - 1));
    const double xl = xs[NIT - 1][i], hl = hs[NIT - 1][i];
    const double rl = hl - eps[(NIT - 1) * N + c] * xl;
    double sx = coef[c * kMaxHist] * xl, sh = coef[c * kMaxHist] * hl, sr = coef[c * kMaxHist] * rl;
#pragma unroll
    for (int k = 0; k < NIT - 1; ++k) {
        const double ck = coef[c * kMaxHist + k + 1];
        const double xk = xs[k][i], hk = hs[k][i];
        sx += ck * (xk - xl);
        sh += ck * (hk - hl);
        sr += ck * ((hk - eps[k * N + c] * xk) - rl);
    }
    xb[i] = (T)sx;
    if (hb != nullptr) hb[i] = (T)sh;
    rb[i] = (T)sr;
}

// ----------------------------------------------------- per-state solvers
// Lowest eigenpair of the symmetric generalised problem A c = mu B c
// (n <= 4): scale by diag(B)^-1/2, Cholesky of B, Jacobi on L^-1 A L^-T.
// Returns false when B is not positive definite.
__device__ bool lowest_geneig(int n, const double *A_in, const double *B_in, double *c) {
    double A[16], Bm[16], D[4], L[16], C[16], V[16];
    for (int i = 0; i < n; ++i) {
        if (!(B_in[i * n + i] > 0.0)) return false;
        D[i] = 1.0 / sqrt(B_in[i * n + i]);
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            A[i * n + j] = A_in[i * n + j] * D[i] * D[j];
            Bm[i * n + j] = B_in[i * n + j] * D[i] * D[j];
        }
    for (int i = 0; i < 16; ++i) L[i] = 0.0;
    for (int j = 0; j < n; ++j) {
        double d = Bm[j * n + j];
        for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
        if (!(d > 0.0)) return false;
        L[j * n + j] = sqrt(d);
        for (int i = j + 1; i < n; ++i) {
            double s = Bm[i * n + j];
            for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = s / L[j * n + j];
        }
    }
    // C = L^-1 A L^-T: solve L Y = A, then L C^T = Y^T
    double Y[16];
    for (int col = 0; col < n; ++col)
        for (int i = 0; i < n; ++i) {
            double s = A[i * n + col];
            for (int k = 0; k < i; ++k) s -= L[i * n + k] * Y[k * n + col];
            Y[i * n + col] = s / L[i * n + i];
        }
    for (int row = 0; row < n; ++row)
        for (int i = 0; i < n; ++i) {
            double s = Y[row * n + i];
            for (int k = 0; k < i; ++k) s -= L[i * n + k] * C[row * n + k];
            C[row * n + i] = s / L[i * n + i];
        }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            V[i * n + j] = i == j ? 1.0 : 0.0;
            if (j > i) C[i * n + j] = C[j * n + i] = 0.5 * (C[i * n + j] + C[j * n + i]);
        }
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += C[i * n + j] * C[i * n + j];
                if (i != j) off += C[i * n + j] * C[i * n + j];
            }
        if (!(off > 1e-32 * tot)) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = C[p * n + q];
                if (apq == 0.0) continue;
                const double th = (C[q * n + q] - C[p * n + p]) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < n; ++k) {
                    const double kp = C[k * n + p], kq = C[k * n + q];
                    C[k * n + p] = cs * kp - sn * kq;
                    C[k * n + q] = sn * kp + cs * kq;
                }
                for (int k = 0; k < n; ++k) {
                    const double pk = C[p * n + k], qk = C[q * n + k];
                    C[p * n + k] = cs * pk - sn * qk;
                    C[q * n + k] = sn * pk + cs * qk;
                }
                for (int k = 0; k < n; ++k) {
                    const double kp = V[k * n + p], kq = V[k * n + q];
                    V[k * n + p] = cs * kp - sn * kq;
                    V[k * n + q] = sn * kp + cs * kq;
                }
            }
    }
    int lo = 0;
    for (int i = 1; i < n; ++i)
        if (C[i * n + i] < C[lo * n + lo]) lo = i;
    // c = D L^-T y
    double y[4];
    for (int i = 0; i < n; ++i) y[i] = V[i * n + lo];
    for (int i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * c[k];
        c[i] = s / L[i * n + i];
    }
    for (int i = 0; i < n; ++i) c[i] *= D[i];
    for (int i = 0; i < n; ++i)
        if (!isfinite(c[i])) return false;
    return true;
}

// Trial step lambda (state frozen -> 0).  dots: [<x|Hx>, <x|x>] and
// [<x|Hd>, <d|Hx>, <d|Hd>, <x|d>, <d|d>].
__global__ void lambda_kernel(const double *__restrict__ d2, const double *__restrict__ d5,
                              const int *__restrict__ active, int N, double *__restrict__ lam) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    double l = 0.0;
    const double b22 = d5[4 * N + c];
    if (active[c] && b22 > 0.0) {
        const double s = 1.0 / sqrt(b22);
        const double a11 = d2[1 * N + c], b11 = d2[0 * N + c];
        const double a12 = 0.5 * (d5[0 * N + c] + d5[1 * N + c]) * s;
        const double a22 = d5[2 * N + c] * s * s;
        const double b12 = d5[3 * N + c] * s;
        const double A[4] = {a11, a12, a12, a22}, Bm[4] = {b11, b12, b12, 1.0};
        double v[2];
        if (lowest_geneig(2, A, Bm, v) && v[0] != 0.0) l = v[1] / v[0] * s;
    }
    lam[c] = l;
}

// Rayleigh quotient of iterate 1 = x + lambda d from the trial-step dots:
// (<x|Hx> + lambda (<x|Hd> + <d|Hx>) + lambda^2 <d|Hd>) /
// (<x|x> + 2 lambda <x|d> + lambda^2 <d|d>).
__global__ void eps1_kernel(const double *__restrict__ d2, const double *__restrict__ d5,
                            const double *__restrict__ lam, int N, double *__restrict__ eps1) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    const double l = lam[c];
    // lambda 0 (frozen states, whose trial-step dots are not formed): iterate
    // 1 is iterate 0
    const double num = l == 0.0 ? d2[1 * N + c]
                                : d2[1 * N + c] + l * (d5[0 * N + c] + d5[1 * N + c]) + l * l * d5[2 * N + c];
    const double den = l == 0.0 ? d2[0 * N + c] : d2[0 * N + c] + 2.0 * l * d5[3 * N + c] + l * l * d5[4 * N + c];
    eps1[c] = den > 0.0 ? num / den : 0.0;
}

// Filter and network coefficients of the trial step (state frozen: lambda
// 0).  d2: [<x|x>, <x|Hx>]; d13: the dots of OpLam3.  The Rayleigh quotient
// is minimised over {x, d/|d|, e/|e|}; the lowest generalised eigenvector,
// first component one, gives mix = (a, b) and lambda = 1.  When that 3x3
// problem is singular the 2x2 filter step is kept: lambda from it, mix =
// (lambda, 0).
__global__ void mix_kernel(const double *__restrict__ d2, const double *__restrict__ d13,
                           const int *__restrict__ active, int N, double *__restrict__ lam,
                           double *__restrict__ mix) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    double l = 0.0, ma = 0.0, mb = 0.0;
    const double bdd = d13[4 * N + c], bee = d13[9 * N + c];
    if (active[c] && bdd > 0.0) {
        const double s = 1.0 / sqrt(bdd);
        const double a11 = d2[1 * N + c], b11 = d2[0 * N + c];
        const double a12 = 0.5 * (d13[0 * N + c] + d13[1 * N + c]) * s;
        const double a22 = d13[2 * N + c] * s * s;
        const double b12 = d13[3 * N + c] * s;
        {
            const double A[4] = {a11, a12, a12, a22}, Bm[4] = {b11, b12, b12, 1.0};
            double v[2];
            if (lowest_geneig(2, A, Bm, v) && v[0] != 0.0) l = v[1] / v[0] * s;
            ma = l;
        }
        if (bee > 0.0 && isfinite(bee)) {
            const double t = 1.0 / sqrt(bee);
            const double a13 = 0.5 * (d13[5 * N + c] + d13[6 * N + c]) * t;
            const double a33 = d13[7 * N + c] * t * t;
            const double b13 = d13[8 * N + c] * t;
            const double a23 = 0.5 * (d13[10 * N + c] + d13[11 * N + c]) * s * t;
            const double b23 = d13[12 * N + c] * s * t;
            const double A[9] = {a11, a12, a13, a12, a22, a23, a13, a23, a33};
            const double Bm[9] = {b11, b12, b13, b12, 1.0, b23, b13, b23, 1.0};
            double v[3];
            if (lowest_geneig(3, A, Bm, v) && v[0] != 0.0) {
                ma = v[1] / v[0] * s;
                mb = v[2] / v[0] * t;
                l = 1.0;
            }
        }
    }
    lam[c] = l;
    mix[c] = ma;
    mix[N + c] = mb;
}

// d = a d + b e (and hd = a hd + b he when given) for the states whose
// network coefficient b is nonzero.
template <typename T>
__global__ void __launch_bounds__(256)
mixdir_kernel(T *__restrict__ d, const T *__restrict__ e, T *__restrict__ hd, const T *__restrict__ he,
              const double *__restrict__ mix, int64_t np, int B, int N, const int *__restrict__ bmap) {
    // blockIdx.y: the block (or its entry in the block map); B is a power of two
    const int blk = bmap ? bmap[blockIdx.y] : (int)blockIdx.y;
    const int64_t il = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (il >= np * B) return;
    const int64_t i = (int64_t)blk * np * B + il;
    const int c = blk * B + (int)(il & (B - 1));
    const double b = mix[N + c];
    if (b == 0.0) return;
    const double a = mix[c];
    d[i] = (T)(a * (double)d[i] + b * (double)e[i]);
    if (hd) hd[i] = (T)(a * (double)hd[i] + b * (double)he[i]);
}

// eps of the newest iterate from its dots [<x|x>, <x|Hx>]
__global__ void eps_kernel(const double *__restrict__ d2, int N, double *__restrict__ eps_out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    const double nn = d2[0 * N + c];
    eps_out[c] = nn > 0.0 ? d2[1 * N + c] / nn : 0.0;     // zero (padding) states: 0
}

// DIIS coefficients per state (c_0 = 1); frozen or degenerate -> e_0.
__global__ void diis_kernel(const double *__restrict__ mats, int n, const double *__restrict__ lam, int N,
                            double *__restrict__ coef) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    double out[kMaxHist] = {1.0, 0.0, 0.0, 0.0};
    if (lam[c] != 0.0) {
        double A[16], Bm[16], v[4];
        const int nt = n * (n + 1) / 2;
        int t = 0;
        for (int p = 0; p < n; ++p)
            for (int q = p; q < n; ++q) {
                A[p * n + q] = A[q * n + p] = mats[(int64_t)t * N + c];
                Bm[p * n + q] = Bm[q * n + p] = mats[(int64_t)(t + nt) * N + c];
                ++t;
            }
        if (lowest_geneig(n, A, Bm, v) && v[0] != 0.0)
            for (int i = 0; i < n; ++i) out[i] = v[i] / v[0];
    }
    for (int i = 0; i < kMaxHist; ++i) coef[c * kMaxHist + i] = out[i];
}

// eps0 = <x|Hx>/<x|x>; after the residual pass: res = sqrt(<R|R>), and a
// block is active unless every state in it is below tol.
// sigma_k = -<psi_k|T psi_k> / <psi_k|psi_k>
__global__ void sigma_kernel(const double *__restrict__ d2, int N, double *__restrict__ sigma) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    const double nn = d2[0 * N + c];
    sigma[c] = nn > 0.0 ? -d2[1 * N + c] / nn : 0.0;
}

__global__ void active_kernel(const double *__restrict__ rr, int N, int B, double tol, int block_stop,
                              double *__restrict__ res, int *__restrict__ active) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    const double r = sqrt(rr[c]);
    res[c] = r;
    int act = 1;
    if (block_stop) {
        const int b0 = (c / B) * B;
        act = 0;
        for (int k = b0; k < b0 + B; ++k) act |= !(sqrt(rr[k]) < tol);
    }
    active[c] = act;
}

}  // namespace

struct rs_solver {
    const rs_grid *g = nullptr;
    const rs_nl *nl = nullptr;
    const void *vloc = nullptr;
    int N = 0, B = 0, nblk = 0, dtype = 0, prec = 0;
    int nreal = 0;                  // states asked for; N - nreal zero padding states
    rs_solver_opts opts{};
    rs_ctx *ctx = nullptr;
    size_t field_bytes = 0;
    rs::DevBuf hx[kMaxHist], hh[kMaxHist];  // history of iterates and H applied
    rs::DevBuf R, d, hd, hpsi;
    rs::DevBuf partial, d2, d5, rr, res, eig, lam, eps, mats, coef, active;
    rs::DevBuf sigma, R0;        // shifts, recorded residuals
    rs::DevBuf dn, hdn;          // network direction and H applied (with a network)
    rs::DevBuf d13, mix;         // trial-subspace dots; filter / network coefficients
    rs::DevBuf bmap;             // int [nblk]: blocks of the trial step and DIIS when some are frozen
    std::vector<int> host_act, host_map;
    rs_cnn *cnn = nullptr;
    int rr_sweeps = kMaxSweeps;
    int steps = 0;
    rs_solver_stats stats{};
};

extern "C" rs_status rs_eigensolve_create(const rs_grid *g, const rs_nl *nl, const void *vloc, int32_t nstates,
                                          int32_t B, int32_t dtype, const rs_solver_opts *opts, rs_solver **out) {
    using namespace rs;
    if (!g || !vloc || !out) return fail(RS_EINVAL, "rs_eigensolve_create: null argument");
    *out = nullptr;
    if (B < 1 || B > 64 || (B & (B - 1))) return fail(RS_EINVAL, "rs_eigensolve_create: bad B");
    if (nstates < 1 || nstates > 256) return fail(RS_EINVAL, "rs_eigensolve_create: nstates must be in [1, 256]");
    if (dtype != RS_F64 && dtype != RS_F32) return fail(RS_EINVAL, "rs_eigensolve_create: bad dtype");
    if (nl && nl->max_states < (nstates + B - 1) / B * B)
        return fail(RS_EINVAL, "rs_eigensolve_create: projector set too small (needs whole blocks)");
    auto s = new (std::nothrow) rs_solver();
    if (!s) return fail(RS_ENOMEM, "host allocation failed");
    s->g = g;
    s->nl = nl;
    s->vloc = vloc;
    s->nblk = (nstates + B - 1) / B;
    s->N = s->nblk * B;               // the last block is padded with zero states
    s->nreal = nstates;
    s->B = B;
    s->dtype = dtype;
    s->prec = dtype == RS_F64 ? RS_PREC_NATIVE : RS_PREC_BF16X3;
    rs_solver_opts o;
    o.m = 3;
    o.alpha = 0.52;
    o.tol = 1e-6;
    o.block_stop = 1;
    o.record = 0;
    o.rr_sweeps = 0;
    if (opts) o = *opts;
    if (o.m < 1 || o.m > kMaxHist - 1) { delete s; return fail(RS_EINVAL, "rs_eigensolve_create: m must be 1..3"); }
    if (o.rr_sweeps < 0 || o.rr_sweeps > kMaxSweeps) {
        delete s;
        return fail(RS_EINVAL, "rs_eigensolve_create: rr_sweeps must be 0..30");
    }
    s->opts = o;
    s->rr_sweeps = o.rr_sweeps ? o.rr_sweeps : kMaxSweeps;
    rs_status st = rs_ctx_create(g, s->N, &s->ctx);
    if (st) { delete s; return st; }
    const size_t es = dtype == RS_F64 ? 8 : 4;
    s->field_bytes = (size_t)g->np * s->N * es;
    const int N = s->N;
    const int nchunks = (int)((g->np + rsred::kChunk - 1) / rsred::kChunk);
    for (int i = 0; i <= o.m && !st; ++i) {   // iterate 0 is the caller's psi
        if (i > 0) st = s->hx[i].alloc(s->field_bytes);
        if (!st) st = s->hh[i].alloc(s->field_bytes);
    }
    if (!st) st = s->R.alloc(s->field_bytes);
    if (!st) st = s->d.alloc(s->field_bytes);
    if (!st) st = s->hd.alloc(s->field_bytes);
    if (!st) st = s->partial.alloc(sizeof(double) * 13 * (size_t)nchunks * N);
    if (!st) st = s->d2.alloc(sizeof(double) * 2 * N);
    if (!st) st = s->d5.alloc(sizeof(double) * 5 * N);
    if (!st) st = s->rr.alloc(sizeof(double) * N);
    if (!st) st = s->res.alloc(sizeof(double) * N);
    if (!st) st = s->eig.alloc(sizeof(double) * N);
    if (!st) st = s->lam.alloc(sizeof(double) * N);
    if (!st) st = s->eps.alloc(sizeof(double) * kMaxHist * N);
    if (!st) st = s->mats.alloc(sizeof(double) * 12 * N);
    if (!st) st = s->coef.alloc(sizeof(double) * kMaxHist * N);
    if (!st) st = s->active.alloc(sizeof(int) * N);
    if (!st) st = s->sigma.alloc(sizeof(double) * N);
    if (!st) st = s->d13.alloc(sizeof(double) * 13 * N);
    if (!st) st = s->mix.alloc(sizeof(double) * 2 * N);
    if (!st) st = s->bmap.alloc(sizeof(int) * s->nblk);
    // reductions over a subset of the blocks leave the other columns'
    // partial sums as they were: start them at zero
    if (!st && hipMemset(s->partial.p, 0, sizeof(double) * 13 * (size_t)nchunks * N) != hipSuccess)
        st = fail(RS_EHIP, "rs_eigensolve_create: clearing the reduction scratch failed");
    if (!st && o.record) st = s->R0.alloc(s->field_bytes);
    if (st) {
        rs_ctx_destroy(s->ctx);
        delete s;
        return st;
    }
    *out = s;
    return RS_OK;
}

extern "C" void rs_eigensolve_destroy(rs_solver *s) {
    if (!s) return;
    rs_ctx_destroy(s->ctx);
    delete s;
}

namespace {

// d = K r for the DIIS iterations: the filter, or per state a K_f r + b K_n r
// with the trial step's coefficients (the network output goes to S->dn).
// The blocks a step's trial and DIIS passes run on: all of them, or, when
// the block stopping rule froze some, the others (map: their indices on the
// device, runs: contiguous ranges for the stencil and network calls, which
// take a first block and a count).
struct Blocks {
    const int *map = nullptr;
    int n = 0;
    std::vector<std::pair<int, int>> runs;
};

// d = K r on the listed blocks: the filter, and with a network its direction
// mixed in per state
template <typename T>
rs_status precond(rs_solver *S, const T *r, T *d, const Blocks &bs, hipStream_t st) {
    using namespace rs;
    const rs_grid *g = S->g;
    const int64_t bel = g->np * S->B;
    for (const auto &run : bs.runs) {
        const int64_t off = run.first * bel;
        rs_status e = filter_apply(g, S->opts.alpha, r + off, d + off, run.second, S->B, S->dtype, st);
        if (e) return e;
        if (S->cnn && (e = cnn_precondition(S->cnn, g, r + off, S->sigma.as<double>() + run.first * S->B,
                                            S->dn.as<T>() + off, run.second, S->B, S->dtype, st)))
            return e;
    }
    if (!S->cnn) return RS_OK;
    const dim3 gb((unsigned)((g->np * S->B + 255) / 256), bs.n);
    hipLaunchKernelGGL(mixdir_kernel<T>, gb, dim3(256), 0, st, d, S->dn.as<T>(), (T *)nullptr, (const T *)nullptr,
                       S->mix.as<double>(), g->np, S->B, S->N, bs.map);
    RS_HIP(hipGetLastError());
    return RS_OK;
}

// H applied to the listed blocks of x
template <typename T>
rs_status hpsi_blocks(rs_solver *S, const T *x, T *hx, const Blocks &bs, hipStream_t st) {
    const int64_t bel = S->g->np * S->B;
    for (const auto &run : bs.runs) {
        const int64_t off = run.first * bel;
        rs_status e = rs::hpsi_apply(S->g, S->nl, S->vloc, x + off, hx + off, run.second, S->B, S->dtype, st);
        if (e) return e;
    }
    return RS_OK;
}

template <typename T>
rs_status step_impl(rs_solver *S, T *psi, hipStream_t st) {
    using namespace rs;
    const rs_grid *g = S->g;
    const int64_t np = g->np;
    const int B = S->B, nblk = S->nblk, N = S->N, m = S->opts.m;
    const double dv = g->h * g->h * g->h;
    const unsigned gs = (unsigned)((N + 63) / 64);
    T *h0 = S->hh[0].as<T>();
    double *partial = S->partial.as<double>();
    rs_status e;
    // 1. H psi, Rayleigh-Ritz
    if ((e = hpsi_apply(g, S->nl, S->vloc, psi, h0, nblk, B, S->dtype, st))) return e;
    if ((e = subspace_diag_capped(S->ctx, psi, h0, S->eig.as<double>(), nblk, B, S->dtype, S->prec, S->rr_sweeps,
                                  S->nreal, st)))
        return e;
    // shifts for the learned preconditioner: sigma = -<psi|T psi>
    if (S->cnn || S->opts.record) {
        if ((e = kinetic_apply(g, psi, S->d.p, nblk, B, S->dtype, st))) return e;
        if ((e = colreduce<2>(OpDots2<T>{psi, S->d.as<T>()}, np, B, nblk, dv, partial, S->d2.as<double>(), st)))
            return e;
        hipLaunchKernelGGL(sigma_kernel, dim3(gs), dim3(64), 0, st, S->d2.as<double>(), N, S->sigma.as<double>());
    }
    // 2. eps0, residual, activity
    if ((e = colreduce<2>(OpDots2<T>{psi, h0}, np, B, nblk, dv, partial, S->d2.as<double>(), st))) return e;
    hipLaunchKernelGGL(eps_kernel, dim3(gs), dim3(64), 0, st, S->d2.as<double>(), N, S->eps.as<double>());
    if ((e = colreduce<1>(OpResid<T>{psi, h0, S->R.as<T>(), S->eps.as<double>()}, np, B, nblk, dv, partial,
                          S->rr.as<double>(), st)))
        return e;
    hipLaunchKernelGGL(active_kernel, dim3(gs), dim3(64), 0, st, S->rr.as<double>(), N, B, S->opts.tol,
                       S->opts.block_stop, S->res.as<double>(), S->active.as<int>());
    if (S->opts.record) RS_HIP(hipMemcpyAsync(S->R0.p, S->R.p, S->field_bytes, hipMemcpyDeviceToDevice, st));
    // Block stopping rule (Sec. 9): the trial step and the DIIS iterations
    // run only on blocks with a state above tolerance; frozen blocks keep
    // psi.  Reading the flags costs one wait on the stream per step, taken
    // only when a block can freeze (block_stop and tol > 0).
    Blocks bs;
    bs.n = nblk;
    bs.runs.assign(1, {0, nblk});
    if (S->opts.block_stop && S->opts.tol > 0.0) {
        S->host_act.resize(N);
        RS_HIP(hipMemcpyAsync(S->host_act.data(), S->active.p, sizeof(int) * N, hipMemcpyDeviceToHost, st));
        RS_HIP(hipStreamSynchronize(st));
        S->host_map.clear();
        for (int b = 0; b < nblk; ++b)
            if (S->host_act[(size_t)b * B]) S->host_map.push_back(b);
        if (S->host_map.empty()) {
            // every block frozen: psi stays; no state mixed a network direction
            if (S->cnn) RS_HIP(hipMemsetAsync(S->mix.p, 0, sizeof(double) * 2 * N, st));
            return RS_OK;
        }
        if ((int)S->host_map.size() < nblk) {
            RS_HIP(hipMemcpyAsync(S->bmap.p, S->host_map.data(), sizeof(int) * S->host_map.size(),
                                  hipMemcpyHostToDevice, st));
            bs.map = S->bmap.as<int>();
            bs.n = (int)S->host_map.size();
            bs.runs.clear();
            for (int i = 0; i < bs.n; ++i) {
                if (i > 0 && S->host_map[i] == S->host_map[i - 1] + 1) ++bs.runs.back().second;
                else bs.runs.push_back({S->host_map[i], 1});
            }
        }
    }
    const dim3 ga((unsigned)((np * B + 255) / 256), bs.n);   // grid over the active blocks (y: map entry)
    // 3. trial step
    for (const auto &run : bs.runs) {
        const int64_t off = run.first * np * B;
        if ((e = filter_apply(g, S->opts.alpha, S->R.as<T>() + off, S->d.as<T>() + off, run.second, B, S->dtype,
                              st)))
            return e;
    }
    if ((e = hpsi_blocks<T>(S, S->d.as<T>(), S->hd.as<T>(), bs, st))) return e;
    if (!S->cnn) {
        if ((e = colreduce<5>(OpLam<T>{psi, h0, S->d.as<T>(), S->hd.as<T>()}, np, B, nblk, dv, partial,
                              S->d5.as<double>(), st, bs.map, bs.n)))
            return e;
        hipLaunchKernelGGL(lambda_kernel, dim3(gs), dim3(64), 0, st, S->d2.as<double>(), S->d5.as<double>(),
                           S->active.as<int>(), N, S->lam.as<double>());
    } else {
        // the network's direction and the 3x3 trial problem; the mixed
        // direction replaces d (and H d) for the states that use it
        for (const auto &run : bs.runs) {
            const int64_t off = run.first * np * B;
            if ((e = cnn_precondition(S->cnn, g, S->R.as<T>() + off, S->sigma.as<double>() + run.first * B,
                                      S->dn.as<T>() + off, run.second, B, S->dtype, st)))
                return e;
        }
        if ((e = hpsi_blocks<T>(S, S->dn.as<T>(), S->hdn.as<T>(), bs, st))) return e;
        if ((e = colreduce<13>(OpLam3<T>{psi, h0, S->d.as<T>(), S->hd.as<T>(), S->dn.as<T>(), S->hdn.as<T>()}, np,
                               B, nblk, dv, partial, S->d13.as<double>(), st, bs.map, bs.n)))
            return e;
        hipLaunchKernelGGL(mix_kernel, dim3(gs), dim3(64), 0, st, S->d2.as<double>(), S->d13.as<double>(),
                           S->active.as<int>(), N, S->lam.as<double>(), S->mix.as<double>());
        hipLaunchKernelGGL(mixdir_kernel<T>, ga, dim3(256), 0, st, S->d.as<T>(), S->dn.as<T>(), S->hd.as<T>(),
                           S->hdn.as<T>(), S->mix.as<double>(), np, B, N, bs.map);
        RS_HIP(hipGetLastError());
    }
    // history: iterate 0 is psi itself
    const T *xs[kMaxHist], *hs[kMaxHist];
    xs[0] = psi;
    hs[0] = h0;
    if (m == 1) {
        // the trial iterate is the newest: straight into psi (in place)
        hipLaunchKernelGGL(axpy1_kernel<T>, ga, dim3(256), 0, st, psi, S->d.as<T>(), psi,
                           S->lam.as<double>(), np, B, bs.map);
        RS_HIP(hipGetLastError());
        return RS_OK;
    }
    // iterate 1: with the filter alone its Rayleigh quotient follows from
    // the trial-step dots and the first DIIS pass writes it; with a network
    // (mixed directions) a pass of its own writes it and its dots
    const bool fused1 = !S->cnn;
    if (fused1) {
        hipLaunchKernelGGL(eps1_kernel, dim3(gs), dim3(64), 0, st, S->d2.as<double>(), S->d5.as<double>(),
                           S->lam.as<double>(), N, S->eps.as<double>() + N);
    } else if ((e = colreduce<2>(OpAxpy2Dots<T>{psi, h0, S->d.as<T>(), S->hd.as<T>(), S->hx[1].as<T>(),
                                               S->hh[1].as<T>(), S->lam.as<double>()},
                                 np, B, nblk, dv, partial, S->d2.as<double>(), st, bs.map, bs.n))) {
        return e;
    }
    xs[1] = S->hx[1].as<T>();
    hs[1] = S->hh[1].as<T>();
    for (int n = 2; n <= m; ++n) {
        // 4. DIIS iteration over the n iterates 0..n-1: eps of the newest
        // (its dots were accumulated when it was written)
        if (n > 2 || !fused1)
            hipLaunchKernelGGL(eps_kernel, dim3(gs), dim3(64), 0, st, S->d2.as<double>(), N,
                               S->eps.as<double>() + (int64_t)(n - 1) * N);
        if (n == 2 && fused1) {
            OpDiis2New<T> op{psi, h0, S->d.as<T>(), S->hd.as<T>(), S->hx[1].as<T>(), S->hh[1].as<T>(),
                             S->lam.as<double>(), S->eps.as<double>(), N};
            if ((e = colreduce<6>(op, np, B, nblk, dv, partial, S->mats.as<double>(), st, bs.map, bs.n))) return e;
        } else if (n == 2) {
            OpDiis<T, 2> op{{xs[0], xs[1]}, {hs[0], hs[1]}, S->eps.as<double>(), N};
            if ((e = colreduce<6>(op, np, B, nblk, dv, partial, S->mats.as<double>(), st, bs.map, bs.n))) return e;
        } else {
            OpDiis<T, 3> op{{xs[0], xs[1], xs[2]}, {hs[0], hs[1], hs[2]}, S->eps.as<double>(), N};
            if ((e = colreduce<12>(op, np, B, nblk, dv, partial, S->mats.as<double>(), st, bs.map, bs.n)))
                return e;
        }
        hipLaunchKernelGGL(diis_kernel, dim3(gs), dim3(64), 0, st, S->mats.as<double>(), n, S->lam.as<double>(), N,
                           S->coef.as<double>());
        // psi_bar, H psi_bar into slot n; R_bar into R.  The last iteration
        // needs no H psi_bar (nothing follows that would use it)
        T *xb = S->hx[n].as<T>(), *hb = n < m ? S->hh[n].as<T>() : nullptr;
        Hist<T> hist{};
        for (int i = 0; i < n; ++i) {
            hist.x[i] = xs[i];
            hist.h[i] = hs[i];
        }
        if (n == 2)
            hipLaunchKernelGGL((combine_kernel<T, 2>), ga, dim3(256), 0, st, hist, S->eps.as<double>(),
                               S->coef.as<double>(), xb, hb, S->R.as<T>(), np, B, N, bs.map);
        else
            hipLaunchKernelGGL((combine_kernel<T, 3>), ga, dim3(256), 0, st, hist, S->eps.as<double>(),
                               S->coef.as<double>(), xb, hb, S->R.as<T>(), np, B, N, bs.map);
        RS_HIP(hipGetLastError());
        if ((e = precond<T>(S, S->R.as<T>(), S->d.as<T>(), bs, st))) return e;
        // H d only where another DIIS iteration follows: the last update
        // needs d alone
        if (n < m && (e = hpsi_blocks<T>(S, S->d.as<T>(), S->hd.as<T>(), bs, st))) return e;
        if (n < m) {
            if ((e = colreduce<2>(OpAxpy2Dots<T>{xb, hb, S->d.as<T>(), S->hd.as<T>(), xb, hb, S->lam.as<double>()},
                                  np, B, nblk, dv, partial, S->d2.as<double>(), st, bs.map, bs.n)))
                return e;
        } else {
            // the newest iterate goes straight into psi; its H psi is not
            // needed
            hipLaunchKernelGGL(axpy1_kernel<T>, ga, dim3(256), 0, st, xb, S->d.as<T>(), psi,
                               S->lam.as<double>(), np, B, bs.map);
        }
        xs[n] = xb;
        hs[n] = hb;
    }
    RS_HIP(hipGetLastError());
    return RS_OK;
}

}  // namespace

extern "C" rs_status rs_eigensolve_step(rs_solver *s, void *psi, double *eig, double *resnorm, int32_t *nconv,
                                        void *stream) {
    using namespace rs;
    if (!s || !psi) return fail(RS_EINVAL, "rs_eigensolve_step: null argument");
    hipStream_t st = (hipStream_t)stream;
    rs_status e = s->dtype == RS_F64 ? step_impl<double>(s, (double *)psi, st) : step_impl<float>(s, (float *)psi, st);
    if (e) return e;
    int32_t info = 0;
    e = orthonormalize_impl(s->ctx, psi, s->nblk, s->B, s->dtype, s->prec, nullptr, &info, s->nreal, st);
    const int n = s->nreal;
    std::vector<double> ev(n), rn(n);
    std::vector<int> act(s->N);
    std::vector<double> mixb(s->cnn ? s->N : 0);
    int sweeps = 0;
    RS_HIP(hipMemcpyAsync(ev.data(), s->eig.p, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    RS_HIP(hipMemcpyAsync(rn.data(), s->res.p, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    RS_HIP(hipMemcpyAsync(act.data(), s->active.p, sizeof(int) * s->N, hipMemcpyDeviceToHost, st));
    RS_HIP(hipMemcpyAsync(&sweeps, ctx_sweeps(s->ctx), sizeof(int), hipMemcpyDeviceToHost, st));
    if (s->cnn)
        RS_HIP(hipMemcpyAsync(mixb.data(), s->mix.as<double>() + s->N, sizeof(double) * s->N, hipMemcpyDeviceToHost,
                              st));
    RS_HIP(hipStreamSynchronize(st));
    s->stats.rr_sweeps = sweeps;
    s->stats.frozen_blocks = 0;
    for (int b = 0; b < s->nblk; ++b) s->stats.frozen_blocks += act[(size_t)b * s->B] == 0;
    s->stats.net_states = 0;
    if (s->cnn)
        for (int k = 0; k < n; ++k) s->stats.net_states += mixb[k] != 0.0;
    if (eig) std::memcpy(eig, ev.data(), sizeof(double) * n);
    if (resnorm) std::memcpy(resnorm, rn.data(), sizeof(double) * n);
    int c = 0;
    for (int k = 0; k < n; ++k) c += rn[k] < s->opts.tol;
    if (nconv) *nconv = c;
    for (int k = 0; k < n; ++k)
        if (!std::isfinite(ev[k]) || !std::isfinite(rn[k]))
            return fail(RS_ENONFINITE, "rs_eigensolve_step: non-finite eigenvalue or residual");
    s->steps++;
    s->stats.steps = s->steps;
    return e;
}

extern "C" rs_status rs_eigensolve_stats(const rs_solver *s, rs_solver_stats *out) {
    if (!s || !out) return rs::fail(RS_EINVAL, "rs_eigensolve_stats: null argument");
    *out = s->stats;
    return RS_OK;
}

extern "C" rs_status rs_eigensolve_set_precond(rs_solver *s, rs_cnn *c) {
    if (!s) return rs::fail(RS_EINVAL, "rs_eigensolve_set_precond: null solver");
    if (c && !s->dn.p) {
        rs_status st = s->dn.alloc(s->field_bytes);
        if (!st) st = s->hdn.alloc(s->field_bytes);
        if (st) return st;
    }
    s->cnn = c;
    return RS_OK;
}

extern "C" rs_status rs_eigensolve_residuals(rs_solver *s, void *R, double *sigma, void *stream) {
    if (!s || !R || !sigma) return rs::fail(RS_EINVAL, "rs_eigensolve_residuals: null argument");
    if (!s->opts.record) return rs::fail(RS_EINVAL, "rs_eigensolve_residuals: the solver was created without record");
    if (s->steps == 0) return rs::fail(RS_EINVAL, "rs_eigensolve_residuals: no step taken yet");
    hipStream_t st = (hipStream_t)stream;
    RS_HIP(hipMemcpyAsync(R, s->R0.p, s->field_bytes, hipMemcpyDeviceToDevice, st));
    RS_HIP(hipMemcpyAsync(sigma, s->sigma.p, sizeof(double) * s->N, hipMemcpyDeviceToDevice, st));
    return RS_OK;
}

extern "C" rs_status rs_eigensolve_orthonormalize(rs_solver *s, void *psi, void *stream) {
    if (!s || !psi) return rs::fail(RS_EINVAL, "rs_eigensolve_orthonormalize: null argument");
    int32_t info = 0;
    return orthonormalize_impl(s->ctx, psi, s->nblk, s->B, s->dtype, s->prec, nullptr, &info, s->nreal,
                               (hipStream_t)stream);
}
