// C ABI of the orthogonalisation / subspace-diagonalisation stage (Sec. 6).
#include <cstring>

#include "dense.hpp"

struct rs_ctx {
    const rs_grid *g = nullptr;
    int max_states = 0;
    rs::DenseWork w;
    rs::DevBuf S, U, T, A, V, ev;   // double [N][N] (ev: [N])
    rs::DevBuf info;                 // int
};

namespace {

rs_status check(const rs_ctx *c, int nblk, int B, int dtype, int prec, const char *who) {
    using rs::fail;
    if (!c) return fail(RS_EINVAL, std::string(who) + ": null context");
    if (B < 1 || B > 64 || (B & (B - 1))) return fail(RS_EINVAL, std::string(who) + ": B must be a power of two in [1, 64]");
    if (nblk < 1 || (int64_t)nblk * B > c->max_states)
        return fail(RS_EINVAL, std::string(who) + ": nblk*B must be in [1, max_states]");
    if (dtype != RS_F64 && dtype != RS_F32) return fail(RS_EINVAL, std::string(who) + ": bad dtype");
    if (prec != RS_PREC_NATIVE && prec != RS_PREC_BF16X3) return fail(RS_EINVAL, std::string(who) + ": bad prec");
    if (dtype == RS_F32 && prec != RS_PREC_BF16X3)
        return fail(RS_ENOTSUP, std::string(who) + ": FP32 fields use RS_PREC_BF16X3 contractions");
    if (dtype == RS_F64 && prec != RS_PREC_NATIVE)
        return fail(RS_ENOTSUP, std::string(who) + ": FP64 fields use RS_PREC_NATIVE contractions");
    return RS_OK;
}

}  // namespace

extern "C" rs_status rs_ctx_create(const rs_grid *g, int32_t max_states, rs_ctx **out) {
    using namespace rs;
    if (!g || !out) return fail(RS_EINVAL, "rs_ctx_create: null argument");
    *out = nullptr;
    if (g->host_only) return fail(RS_EINVAL, "rs_ctx_create: host-only grid");
    if (max_states < 1 || max_states > 256) return fail(RS_EINVAL, "rs_ctx_create: max_states must be in [1, 256]");
    auto c = new (std::nothrow) rs_ctx();
    if (!c) return fail(RS_ENOMEM, "host allocation failed");
    c->g = g;
    c->max_states = max_states;
    const size_t nn = (size_t)max_states * max_states * sizeof(double);
    rs_status s = dense_work_init(c->w, g->np, max_states);
    if (!s) s = c->S.alloc(nn);
    if (!s) s = c->U.alloc(nn);
    if (!s) s = c->T.alloc(nn);
    if (!s) s = c->A.alloc(nn);
    if (!s) s = c->V.alloc(nn);
    if (!s) s = c->ev.alloc(max_states * sizeof(double));
    if (!s) s = c->info.alloc(sizeof(int));
    if (s) { delete c; return s; }
    *out = c;
    return RS_OK;
}

extern "C" void rs_ctx_destroy(rs_ctx *c) { delete c; }

// Jacobi sweeps of the context's last symmetric eigensolve (device int).
const int *ctx_sweeps(const rs_ctx *c) { return c->w.sweeps.as<int>(); }

extern "C" rs_status rs_overlap(rs_ctx *c, const void *x, const void *y, double *S, int32_t nblk, int32_t B,
                                int32_t dtype, int32_t prec, void *stream) {
    // complex states: the real product of the 2N interleaved columns, then
    // the fold into the Hermitian N x N matrix
    const bool cplx = dtype == RS_C128 || dtype == RS_C64;
    if (cplx) {
        if (B > 32) return rs::fail(RS_EINVAL, "rs_overlap: complex blocks hold at most 32 states");
        dtype = dtype == RS_C128 ? RS_F64 : RS_F32;
        B *= 2;
    }
    rs_status st = check(c, nblk, B, dtype, prec, "rs_overlap");
    if (st) return st;
    if (!x || !y || !S) return rs::fail(RS_EINVAL, "rs_overlap: null pointer");
    const double dv = c->g->h * c->g->h * c->g->h;
    const hipStream_t s = (hipStream_t)stream;
    if (!cplx) return rs::gram(c->w, x, y, c->g->np, B, nblk, dtype, prec, dv, S, 0, s);
    if ((st = rs::gram(c->w, x, y, c->g->np, B, nblk, dtype, prec, dv, c->A.as<double>(), 0, s))) return st;
    return rs::complex_fold(c->A.as<double>(), S, nblk * B / 2, s);
}

extern "C" rs_status rs_rotate(rs_ctx *c, void *psi, const double *X, int32_t nblk, int32_t B, int32_t dtype,
                               int32_t prec, void *stream) {
    rs_status st = check(c, nblk, B, dtype, prec, "rs_rotate");
    if (st) return st;
    if (!psi || !X) return rs::fail(RS_EINVAL, "rs_rotate: null pointer");
    return rs::rotate(c->w, psi, X, c->g->np, B, nblk, dtype, prec, nullptr, (hipStream_t)stream);
}

extern "C" rs_status rs_cholesky(rs_ctx *c, const double *S, double *U, int32_t N, int32_t *info, void *stream) {
    if (!c || !S || !U || !info) return rs::fail(RS_EINVAL, "rs_cholesky: null argument");
    if (N < 1 || N > c->max_states) return rs::fail(RS_EINVAL, "rs_cholesky: N out of range");
    return rs::cholesky(c->w, S, U, N, info, (hipStream_t)stream);
}

extern "C" rs_status rs_eigh(rs_ctx *c, double *A, double *V, double *evals, int32_t N, void *stream) {
    if (!c || !A || !V || !evals) return rs::fail(RS_EINVAL, "rs_eigh: null argument");
    if (N < 1 || N > c->max_states) return rs::fail(RS_EINVAL, "rs_eigh: N out of range");
    return rs::eigh(c->w, A, V, evals, N, (hipStream_t)stream);
}

// nreal < nblk * B: the states from nreal on are zero padding (they get an
// identity pivot and stay zero).
rs_status orthonormalize_impl(rs_ctx *c, void *psi, int nblk, int B, int dtype, int prec, double *S_out,
                              int32_t *info, int nreal, hipStream_t s) {
    rs_status st = check(c, nblk, B, dtype, prec, "rs_orthonormalize_block");
    if (st) return st;
    if (!psi) return rs::fail(RS_EINVAL, "rs_orthonormalize_block: null psi");
    const int N = nblk * B;
    const double dv = c->g->h * c->g->h * c->g->h;
    double *S = S_out ? S_out : c->S.as<double>();
    if ((st = rs::gram(c->w, psi, psi, c->g->np, B, nblk, dtype, prec, dv, S, 0, s))) return st;
    if ((st = rs::pad_identity(S, N, nreal, s))) return st;
    if ((st = rs::cholesky(c->w, S, c->U.as<double>(), N, c->info.as<int>(), s))) return st;
    if ((st = rs::trinv(c->U.as<double>(), c->T.as<double>(), N, c->info.as<int>(), s))) return st;
    if ((st = rs::rotate(c->w, psi, c->T.as<double>(), c->g->np, B, nblk, dtype, prec, c->info.as<int>(), s,
                         true)))
        return st;
    int h_info = 0;
    RS_HIP(hipMemcpyAsync(&h_info, c->info.p, sizeof(int), hipMemcpyDeviceToHost, s));
    RS_HIP(hipStreamSynchronize(s));
    if (info) *info = h_info;
    if (h_info) return rs::fail(RS_ENOTPOSDEF, "rs_orthonormalize_block: overlap not positive definite at column " +
                                                   std::to_string(h_info));
    return RS_OK;
}

extern "C" rs_status rs_orthonormalize_block(rs_ctx *c, void *psi, int32_t nblk, int32_t B, int32_t dtype,
                                             int32_t prec, double *S_out, int32_t *info, void *stream) {
    return orthonormalize_impl(c, psi, nblk, B, dtype, prec, S_out, info, nblk * B, (hipStream_t)stream);
}

rs_status subspace_diag_capped(rs_ctx *c, void *psi, void *hpsi, double *eig, int nblk, int B, int dtype,
                               int prec, int max_sweeps, int nreal, hipStream_t s) {
    rs_status st = check(c, nblk, B, dtype, prec, "rs_subspace_diag");
    if (st) return st;
    if (!psi || !hpsi || !eig) return rs::fail(RS_EINVAL, "rs_subspace_diag: null pointer");
    const int N = nblk * B;
    const double dv = c->g->h * c->g->h * c->g->h;
    if ((st = rs::gram(c->w, psi, hpsi, c->g->np, B, nblk, dtype, prec, dv, c->A.as<double>(), 2, s))) return st;
    if ((st = rs::eigh_leading(c->w, c->A.as<double>(), c->V.as<double>(), eig, N, nreal, c->S.as<double>(),
                               c->U.as<double>(), s, max_sweeps)))
        return st;
    if ((st = rs::rotate(c->w, psi, c->V.as<double>(), c->g->np, B, nblk, dtype, prec, nullptr, s))) return st;
    return rs::rotate(c->w, hpsi, c->V.as<double>(), c->g->np, B, nblk, dtype, prec, nullptr, s);
}

extern "C" rs_status rs_subspace_diag(rs_ctx *c, void *psi, void *hpsi, double *eig, int32_t nblk, int32_t B,
                                      int32_t dtype, int32_t prec, void *stream) {
    return subspace_diag_capped(c, psi, hpsi, eig, nblk, B, dtype, prec, 30, nblk * B, (hipStream_t)stream);
}

