// The self-consistent field loop (Sec. 3, Fig. "groundstate") on the GPU.
//
// One iteration: V_eff = V_ion + V_H[n_in] + V_xc[n_in] (the Hartree
// potential by the FFT solve of Sec. 7, the local density approximation for
// exchange-correlation); a fixed number of RMM-DIIS steps on the states with
// that potential; n_out = 2 sum_{k < nocc} psi_k^2 (eq. 1b, closed shell,
// real states); F = n_out - n_in; Broyden's second method in Anderson's
// form: gamma minimises ||F - sum_j gamma_j dF_j|| over the differences of
// the last m iterations, n_in' = n_in + a F - sum_j gamma_j (dn_j + a dF_j).
// Densities, potentials and the mixing history are FP64 vectors over the
// grid's inner points; every inner product is a fixed-order two-stage sum.
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace {

constexpr int kMaxHistory = 8;
constexpr int kDotBlocks = 512;    // partial sums of a dot product

// Perdew-Zunger (1981) unpolarised correlation constants
constexpr double kPzGamma = -0.1423, kPzBeta1 = 1.0529, kPzBeta2 = 0.3334;
constexpr double kPzA = 0.0311, kPzB = -0.048, kPzC = 0.0020, kPzD = -0.0116;

// n[p] = 2 sum_{k < nocc} psi_k(p)^2, psi in blocks [blk][np][B]
template <typename T>
__global__ void __launch_bounds__(256)
density_kernel(const T *__restrict__ psi, int64_t np, int B, int nocc, double *__restrict__ n) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= np) return;
    double s = 0.0;
    for (int k = 0; k < nocc; ++k) {
        const double v = psi[(int64_t)(k / B) * np * B + p * B + (k % B)];
        s += v * v;
    }
    n[p] = 2.0 * s;
}

// v_xc of the local density approximation (Dirac exchange, Perdew-Zunger
// correlation); zero where n <= 0.
__device__ double lda_vxc(double n) {
    if (!(n > 0.0)) return 0.0;
    const double c13 = cbrt(3.0 * n / M_PI);
    const double vx = -c13;
    const double rs = cbrt(3.0 / (4.0 * M_PI * n));
    double vc;
    if (rs >= 1.0) {
        const double sr = sqrt(rs);
        const double den = 1.0 + kPzBeta1 * sr + kPzBeta2 * rs;
        const double ec = kPzGamma / den;
        vc = ec * (1.0 + (7.0 / 6.0) * kPzBeta1 * sr + (4.0 / 3.0) * kPzBeta2 * rs) / den;
    } else {
        const double lr = log(rs);
        vc = kPzA * lr + (kPzB - kPzA / 3.0) + (2.0 / 3.0) * kPzC * rs * lr + (2.0 * kPzD - kPzC) / 3.0 * rs;
    }
    return vx + vc;
}

template <typename T>
__global__ void __launch_bounds__(256)
veff_kernel(const double *__restrict__ vion, const double *__restrict__ vh, const double *__restrict__ n,
            int64_t np, T *__restrict__ veff) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < np) veff[p] = (T)((vion[p] + vh[p]) + lda_vxc(n[p]));
}

// y = x - w (elementwise)
__global__ void __launch_bounds__(256)
sub_kernel(const double *__restrict__ x, const double *__restrict__ w, int64_t np, double *__restrict__ y) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < np) y[p] = x[p] - w[p];
}

// partial[b] = sum over block b's strided points of x y (fixed order)
__global__ void __launch_bounds__(256)
dot_partial_kernel(const double *__restrict__ x, const double *__restrict__ y, int64_t np, double *__restrict__ part) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < np; p += (int64_t)kDotBlocks * 256)
        s += x[p] * y[p];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out = dv * sum of the partials (one wave, fixed butterfly)
__global__ void __launch_bounds__(64) dot_final_kernel(const double *__restrict__ part, double dv, double *__restrict__ out) {
    double s = 0.0;
    for (int b = threadIdx.x; b < kDotBlocks; b += 64) s += part[b];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (threadIdx.x == 0) *out = dv * s;
}

// gamma from A gamma = b (the Gram matrix of the dF_j and their products
// with F), Gaussian elimination with partial pivoting; a singular system
// gives gamma = 0 (plain linear mixing this iteration).
__global__ void gamma_kernel(const double *__restrict__ gram, int m, double *__restrict__ gamma) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double A[kMaxHistory][kMaxHistory + 1];
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < m; ++j) A[i][j] = gram[i * (m + 1) + j];
        A[i][m] = gram[i * (m + 1) + m];
    }
    bool ok = true;
    for (int c = 0; c < m && ok; ++c) {
        int piv = c;
        for (int r = c + 1; r < m; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        if (!(fabs(A[piv][c]) > 1e-300)) { ok = false; break; }
        if (piv != c)
            for (int j = 0; j <= m; ++j) { const double t = A[c][j]; A[c][j] = A[piv][j]; A[piv][j] = t; }
        for (int r = c + 1; r < m; ++r) {
            const double f = A[r][c] / A[c][c];
            for (int j = c; j <= m; ++j) A[r][j] -= f * A[c][j];
        }
    }
    double g[kMaxHistory];
    for (int i = m - 1; i >= 0 && ok; --i) {
        double s = A[i][m];
        for (int j = i + 1; j < m; ++j) s -= A[i][j] * g[j];
        g[i] = s / A[i][i];
        if (!isfinite(g[i])) ok = false;
    }
    for (int i = 0; i < m; ++i) gamma[i] = ok ? g[i] : 0.0;
}

struct MixHist {
    const double *dn[kMaxHistory], *dF[kMaxHistory];
};

// n_in <- n_in + a F - sum_j gamma_j (dn_j + a dF_j)
__global__ void __launch_bounds__(256)
mix_kernel(double *__restrict__ n_in, const double *__restrict__ F, MixHist h, const double *__restrict__ gamma,
           int m, double a, int64_t np) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= np) return;
    double v = n_in[p] + a * F[p];
    for (int j = 0; j < m; ++j) v -= gamma[j] * (h.dn[j][p] + a * h.dF[j][p]);
    n_in[p] = v;
}

}  // namespace

struct rs_scf {
    const rs_grid *g = nullptr;
    int dtype = 0, nstates = 0, B = 0, nblk = 0;
    rs_scf_opts opts{};
    rs_solver *solver = nullptr;
    rs_poisson *poisson = nullptr;
    rs::DevBuf vion, vh, veff, n_in, n_out, F, prev_n, prev_F, part, gram, gamma;
    rs::DevBuf dn[kMaxHistory], dF[kMaxHistory];
    int nhist = 0, head = 0;        // ring of the last nhist differences; head = next slot
    bool have_prev = false, started = false;
    int iters = 0;
};

namespace {

rs_status dot(rs_scf *s, const double *x, const double *y, double *out, hipStream_t st) {
    hipLaunchKernelGGL(dot_partial_kernel, dim3(kDotBlocks), dim3(256), 0, st, x, y, s->g->np, s->part.as<double>());
    RS_HIP(hipGetLastError());
    const double dv = s->g->h * s->g->h * s->g->h;
    hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(64), 0, st, s->part.as<double>(), dv, out);
    RS_HIP(hipGetLastError());
    return RS_OK;
}

rs_status compute_density(rs_scf *s, const void *psi, double *n, hipStream_t st) {
    const int64_t np = s->g->np;
    const dim3 grid((unsigned)((np + 255) / 256));
    if (s->dtype == RS_F64)
        hipLaunchKernelGGL(density_kernel<double>, grid, dim3(256), 0, st, (const double *)psi, np, s->B, s->opts.nocc, n);
    else
        hipLaunchKernelGGL(density_kernel<float>, grid, dim3(256), 0, st, (const float *)psi, np, s->B, s->opts.nocc, n);
    RS_HIP(hipGetLastError());
    return RS_OK;
}

}  // namespace

extern "C" rs_status rs_scf_create(const rs_grid *g, const rs_nl *nl, const double *vion, int32_t nstates, int32_t B,
                                   int32_t dtype, const rs_scf_opts *opts, rs_scf **out) {
    using rs::fail;
    if (!g || !vion || !opts || !out) return fail(RS_EINVAL, "rs_scf_create: null argument");
    *out = nullptr;
    if (opts->nocc < 1 || opts->nocc > nstates) return fail(RS_EINVAL, "rs_scf_create: nocc must be in [1, nstates]");
    if (opts->eig_steps < 1 || opts->eig_steps > 100) return fail(RS_EINVAL, "rs_scf_create: eig_steps must be 1..100");
    if (opts->history < 0 || opts->history > kMaxHistory) return fail(RS_EINVAL, "rs_scf_create: history must be 0..8");
    if (!(opts->mix > 0.0 && opts->mix <= 1.0)) return fail(RS_EINVAL, "rs_scf_create: mix must be in (0, 1]");
    auto s = new (std::nothrow) rs_scf();
    if (!s) return fail(RS_ENOMEM, "host allocation failed");
    s->g = g;
    s->dtype = dtype;
    s->nstates = nstates;
    s->B = B;
    s->nblk = (nstates + B - 1) / B;
    s->opts = *opts;
    const size_t vb = sizeof(double) * (size_t)g->np;
    rs_status st = RS_OK;
    if (!st) st = s->vion.alloc(vb);
    if (!st) st = s->vh.alloc(vb);
    if (!st) st = s->veff.alloc((dtype == RS_F64 ? 8 : 4) * (size_t)g->np);
    if (!st) st = s->n_in.alloc(vb);
    if (!st) st = s->n_out.alloc(vb);
    if (!st) st = s->F.alloc(vb);
    if (!st) st = s->prev_n.alloc(vb);
    if (!st) st = s->prev_F.alloc(vb);
    for (int j = 0; j < opts->history && !st; ++j) {
        st = s->dn[j].alloc(vb);
        if (!st) st = s->dF[j].alloc(vb);
    }
    if (!st) st = s->part.alloc(sizeof(double) * kDotBlocks);
    if (!st) st = s->gram.alloc(sizeof(double) * (kMaxHistory * (kMaxHistory + 1) + 1));
    if (!st) st = s->gamma.alloc(sizeof(double) * kMaxHistory);
    if (!st) st = rs_poisson_create(g, &s->poisson);
    if (!st) st = rs_eigensolve_create(g, nl, s->veff.p, nstates, B, dtype, &opts->solver, &s->solver);
    if (!st && hipMemcpy(s->vion.p, vion, vb, hipMemcpyDeviceToDevice) != hipSuccess)
        st = fail(RS_EHIP, "rs_scf_create: copy of the ionic potential failed");
    if (st) {
        rs_scf_destroy(s);
        return st;
    }
    *out = s;
    return RS_OK;
}

extern "C" void rs_scf_destroy(rs_scf *s) {
    if (!s) return;
    if (s->solver) rs_eigensolve_destroy(s->solver);
    if (s->poisson) rs_poisson_destroy(s->poisson);
    delete s;
}

extern "C" rs_status rs_scf_start(rs_scf *s, void *psi, void *stream) {
    if (!s || !psi) return rs::fail(RS_EINVAL, "rs_scf_start: null argument");
    hipStream_t st = (hipStream_t)stream;
    rs_status e = rs_eigensolve_orthonormalize(s->solver, psi, stream);
    if (e) return e;
    if ((e = compute_density(s, psi, s->n_in.as<double>(), st))) return e;
    s->nhist = s->head = 0;
    s->have_prev = false;
    s->started = true;
    s->iters = 0;
    return RS_OK;
}

extern "C" rs_status rs_scf_iterate(rs_scf *s, void *psi, double *eig, double *resnorm, double *dens_res,
                                    void *stream) {
    using namespace rs;
    if (!s || !psi) return fail(RS_EINVAL, "rs_scf_iterate: null argument");
    if (!s->started) return fail(RS_EINVAL, "rs_scf_iterate: call rs_scf_start first");
    hipStream_t st = (hipStream_t)stream;
    const int64_t np = s->g->np;
    const dim3 grid((unsigned)((np + 255) / 256));
    // 1. effective potential of n_in
    rs_status e = rs_poisson_solve(s->poisson, s->n_in.as<double>(), s->vh.as<double>(), stream);
    if (e) return e;
    if (s->dtype == RS_F64)
        hipLaunchKernelGGL(veff_kernel<double>, grid, dim3(256), 0, st, s->vion.as<double>(), s->vh.as<double>(),
                           s->n_in.as<double>(), np, s->veff.as<double>());
    else
        hipLaunchKernelGGL(veff_kernel<float>, grid, dim3(256), 0, st, s->vion.as<double>(), s->vh.as<double>(),
                           s->n_in.as<double>(), np, s->veff.as<float>());
    RS_HIP(hipGetLastError());
    // 2. eigensolver steps
    for (int k = 0; k < s->opts.eig_steps; ++k) {
        int32_t nconv = 0;
        if ((e = rs_eigensolve_step(s->solver, psi, eig, resnorm, &nconv, stream))) return e;
    }
    // 3. output density and its distance from the input
    if ((e = compute_density(s, psi, s->n_out.as<double>(), st))) return e;
    hipLaunchKernelGGL(sub_kernel, grid, dim3(256), 0, st, s->n_out.as<double>(), s->n_in.as<double>(), np,
                       s->F.as<double>());
    RS_HIP(hipGetLastError());
    double *gram = s->gram.as<double>();
    double *ff = gram + kMaxHistory * (kMaxHistory + 1);
    if ((e = dot(s, s->F.as<double>(), s->F.as<double>(), ff, st))) return e;
    // 4. mixing: push the differences to the previous iteration, then solve
    //    for gamma over the ring (oldest first)
    const int M = s->opts.history;
    if (s->have_prev && M > 0) {
        hipLaunchKernelGGL(sub_kernel, grid, dim3(256), 0, st, s->n_in.as<double>(), s->prev_n.as<double>(), np,
                           s->dn[s->head].as<double>());
        hipLaunchKernelGGL(sub_kernel, grid, dim3(256), 0, st, s->F.as<double>(), s->prev_F.as<double>(), np,
                           s->dF[s->head].as<double>());
        RS_HIP(hipGetLastError());
        s->head = (s->head + 1) % M;
        s->nhist = std::min(s->nhist + 1, M);
    }
    RS_HIP(hipMemcpyAsync(s->prev_n.p, s->n_in.p, sizeof(double) * np, hipMemcpyDeviceToDevice, st));
    RS_HIP(hipMemcpyAsync(s->prev_F.p, s->F.p, sizeof(double) * np, hipMemcpyDeviceToDevice, st));
    s->have_prev = true;
    const int m = s->nhist;
    MixHist h{};
    for (int j = 0; j < m; ++j) {
        const int slot = (s->head - m + j + 2 * M) % M;     // oldest first
        h.dn[j] = s->dn[slot].as<double>();
        h.dF[j] = s->dF[slot].as<double>();
    }
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < m; ++j)
            if ((e = dot(s, h.dF[i], h.dF[j], gram + i * (m + 1) + j, st))) return e;
        if ((e = dot(s, h.dF[i], s->F.as<double>(), gram + i * (m + 1) + m, st))) return e;
    }
    if (m > 0) {
        hipLaunchKernelGGL(gamma_kernel, dim3(1), dim3(64), 0, st, gram, m, s->gamma.as<double>());
        RS_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(mix_kernel, grid, dim3(256), 0, st, s->n_in.as<double>(), s->F.as<double>(), h,
                       s->gamma.as<double>(), m, s->opts.mix, np);
    RS_HIP(hipGetLastError());
    double ffh = 0.0;
    RS_HIP(hipMemcpyAsync(&ffh, ff, sizeof(double), hipMemcpyDeviceToHost, st));
    RS_HIP(hipStreamSynchronize(st));
    if (dens_res) *dens_res = std::sqrt(ffh);
    s->iters++;
    return RS_OK;
}

extern "C" rs_status rs_scf_density(const rs_scf *s, double *n_in, double *n_out, void *stream) {
    if (!s) return rs::fail(RS_EINVAL, "rs_scf_density: null handle");
    hipStream_t st = (hipStream_t)stream;
    const size_t b = sizeof(double) * (size_t)s->g->np;
    if (n_in) RS_HIP(hipMemcpyAsync(n_in, s->n_in.p, b, hipMemcpyDeviceToDevice, st));
    if (n_out) RS_HIP(hipMemcpyAsync(n_out, s->n_out.p, b, hipMemcpyDeviceToDevice, st));
    return RS_OK;
}
