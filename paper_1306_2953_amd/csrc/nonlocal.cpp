// Host construction of the Kleinman-Bylander projector set (eq. (6),
// Sec. 5.3): per-atom sphere point lists, the values of the (l_max+1)^2
// projectors gamma_lm = N_l r^l Y_lm exp(-r^2 / 2 sigma^2) (real spherical
// harmonics, l = 0..l_max <= 3), colour groups,
// the chunked work list of the projection kernel and the point-centric table
// of the fused apply.  Built with -ffp-contract=off so that sphere
// membership, |r_p - R_A|^2 = ((dx*dx + dy*dy) + dz*dz) <= rc*rc, is decided
// by exactly rounded operations.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.hpp"

namespace {

constexpr int kChunk = 512;   // sphere entries per projection work-group

double min_image(double d, double L) { return d - L * std::nearbyint(d / L); }

// Projector values at displacement d (r2 = |d|^2 formed as (dx dx + dy dy)
// + dz dz, e = exp(-r2 / 2 sigma^2)) into out[(lmax+1)^2]: l ascending; l = 1
// in the order x, y, z; l = 2: xy, yz, 3z^2 - r^2, xz, x^2 - y^2; l = 3:
// y(3x^2 - y^2), xyz, y(5z^2 - r^2), z(5z^2 - 3r^2), x(5z^2 - r^2),
// z(x^2 - y^2), x(x^2 - 3y^2).  nrm[l] = N_l times the harmonic's
// constant is applied per function; l <= 1 uses N_s and N_p directly.
struct ProjectorShape {
    int lmax;
    double ns, npn;      // N_0 Y_00 and N_1 sqrt(3 / 4 pi)
    double c2[3];        // N_2 times 1/2 sqrt(15/pi), 1/4 sqrt(5/pi), 1/4 sqrt(15/pi)
    double c3[5];        // N_3 times 1/4 sqrt(35/2pi), 1/2 sqrt(105/pi), 1/4 sqrt(21/2pi),
                         //           1/4 sqrt(7/pi), 1/4 sqrt(105/pi)

    ProjectorShape(int lmax_, double sigma) : lmax(lmax_) {
        const double pi = 3.14159265358979323846;
        ns = 1.0 / std::sqrt(std::pow(pi, 1.5) * sigma * sigma * sigma);
        npn = 1.0 / std::sqrt(std::pow(pi, 1.5) * std::pow(sigma, 5) / 2.0);
        // N_l = (Gamma(l + 3/2) sigma^(2l+3) / 2)^(-1/2)
        const double n2 = 1.0 / std::sqrt(std::tgamma(3.5) * std::pow(sigma, 7) / 2.0);
        const double n3 = 1.0 / std::sqrt(std::tgamma(4.5) * std::pow(sigma, 9) / 2.0);
        c2[0] = n2 * 0.5 * std::sqrt(15.0 / pi);
        c2[1] = n2 * 0.25 * std::sqrt(5.0 / pi);
        c2[2] = n2 * 0.25 * std::sqrt(15.0 / pi);
        c3[0] = n3 * 0.25 * std::sqrt(35.0 / (2.0 * pi));
        c3[1] = n3 * 0.5 * std::sqrt(105.0 / pi);
        c3[2] = n3 * 0.25 * std::sqrt(21.0 / (2.0 * pi));
        c3[3] = n3 * 0.25 * std::sqrt(7.0 / pi);
        c3[4] = n3 * 0.25 * std::sqrt(105.0 / pi);
    }

    void eval(const double d[3], double r2, double e, double *out) const {
        const double x = d[0], y = d[1], z = d[2];
        out[0] = ns * e;
        if (lmax < 1) return;
        out[1] = npn * x * e;
        out[2] = npn * y * e;
        out[3] = npn * z * e;
        if (lmax < 2) return;
        out[4] = c2[0] * x * y * e;
        out[5] = c2[0] * y * z * e;
        out[6] = c2[1] * (3.0 * z * z - r2) * e;
        out[7] = c2[0] * x * z * e;
        out[8] = c2[2] * (x * x - y * y) * e;
        if (lmax < 3) return;
        out[9] = c3[0] * y * (3.0 * x * x - y * y) * e;
        out[10] = c3[1] * x * y * z * e;
        out[11] = c3[2] * y * (5.0 * z * z - r2) * e;
        out[12] = c3[3] * z * (5.0 * z * z - 3.0 * r2) * e;
        out[13] = c3[2] * x * (5.0 * z * z - r2) * e;
        out[14] = c3[4] * z * (x * x - y * y) * e;
        out[15] = c3[0] * x * (x * x - 3.0 * y * y) * e;
    }
};

}  // namespace

extern "C" rs_status rs_nl_create(const rs_grid *g, int32_t nat, const double *pos,
                                  const double *D, double rc, double sigma, int32_t lmax,
                                  int32_t max_states, rs_nl **out) {
    using namespace rs;
    if (!g || !out) return fail(RS_EINVAL, "rs_nl_create: null argument");
    *out = nullptr;
    if (nat < 0 || (nat > 0 && (!pos || !D))) return fail(RS_EINVAL, "rs_nl_create: bad atoms");
    if (!(rc > 0) || !(sigma > 0)) return fail(RS_EINVAL, "rs_nl_create: rc and sigma must be > 0");
    if (lmax < 0 || lmax > 3) return fail(RS_EINVAL, "rs_nl_create: lmax must be 0..3");
    if (max_states < 1 || max_states > 4096) return fail(RS_EINVAL, "rs_nl_create: max_states out of range");
    auto nl = new (std::nothrow) rs_nl();
    if (!nl) return fail(RS_ENOMEM, "host allocation failed");
    nl->nat = nat;
    nl->lmax = lmax;
    nl->npj = (lmax + 1) * (lmax + 1);
    const int npj = nl->npj;
    nl->max_states = max_states;
    nl->dv = g->h * g->h * g->h;
    nl->D.assign(D, D + npj * (size_t)nat);

    const bool periodic = g->kind == RS_GRID_PERIODIC;
    const double Lbox = periodic ? (double)g->n * g->h : 0.0;
    const double rc2 = rc * rc;
    const ProjectorShape shape(lmax, sigma);
    const double inv2s2 = 1.0 / (2.0 * sigma * sigma);

    nl->sph_ptr.assign(nat + 1, 0);
    const int64_t R = (int64_t)std::ceil(rc / g->h) + 1;
    for (int A = 0; A < nat; ++A) {
        const double X[3] = {pos[3 * A], pos[3 * A + 1], pos[3 * A + 2]};
        std::vector<int64_t> pts;
        auto consider = [&](int64_t p) {
            double d[3];
            for (int a = 0; a < 3; ++a) {
                d[a] = ((double)g->inner[3 * p + a] - g->centre) * g->h - X[a];
                if (periodic) d[a] = min_image(d[a], Lbox);
            }
            const double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
            if (r2 <= rc2) pts.push_back(p);
        };
        if (periodic && 2 * R + 1 > g->n) {
            for (int64_t p = 0; p < g->np; ++p) consider(p);
        } else {
            int64_t c[3];
            for (int a = 0; a < 3; ++a) c[a] = (int64_t)std::floor(X[a] / g->h + g->centre + 0.5);
            for (int64_t k = c[2] - R; k <= c[2] + R; ++k)
                for (int64_t j = c[1] - R; j <= c[1] + R; ++j)
                    for (int64_t i = c[0] - R; i <= c[0] + R; ++i) {
                        int64_t ii = i, jj = j, kk = k;
                        if (periodic) {
                            ii = ((ii % g->n) + g->n) % g->n;
                            jj = ((jj % g->n) + g->n) % g->n;
                            kk = ((kk % g->n) + g->n) % g->n;
                        }
                        if (ii < g->lo[0] || jj < g->lo[1] || kk < g->lo[2] ||
                            ii >= g->lo[0] + g->L[0] || jj >= g->lo[1] + g->L[1] ||
                            kk >= g->lo[2] + g->L[2])
                            continue;
                        const int64_t p = g->lookup[g->lattice_index(ii, jj, kk)];
                        if (p >= 0) consider(p);
                    }
        }
        std::sort(pts.begin(), pts.end());
        for (int64_t p : pts) {
            double d[3];
            for (int a = 0; a < 3; ++a) {
                d[a] = ((double)g->inner[3 * p + a] - g->centre) * g->h - X[a];
                if (periodic) d[a] = min_image(d[a], Lbox);
            }
            const double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
            const double e = std::exp(-r2 * inv2s2);
            double val[16];
            shape.eval(d, r2, e, val);
            nl->sph_idx.push_back(p);
            nl->gamma.insert(nl->gamma.end(), val, val + npj);
        }
        nl->sph_ptr[A + 1] = (int64_t)nl->sph_idx.size();
    }
    const int64_t nnz = (int64_t)nl->sph_idx.size();

    // greedy colouring in atom order: smallest colour unused by earlier
    // atoms whose spheres overlap (|R_A - R_B| <= 2 rc)
    nl->colour.assign(nat, 0);
    const double lim = (2.0 * rc) * (2.0 * rc);
    for (int A = 0; A < nat; ++A) {
        std::vector<char> used(nat + 1, 0);
        for (int Bq = 0; Bq < A; ++Bq) {
            double d[3];
            for (int a = 0; a < 3; ++a) {
                d[a] = pos[3 * A + a] - pos[3 * Bq + a];
                if (periodic) d[a] = min_image(d[a], Lbox);
            }
            if ((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2] <= lim) used[nl->colour[Bq]] = 1;
        }
        int c = 0;
        while (used[c]) ++c;
        nl->colour[A] = c;
        nl->ncolours = std::max(nl->ncolours, c + 1);
    }

    // chunked work list for the projections
    std::vector<int32_t> ch_atom, ch_beg, ch_end, atom_chunk0(nat + 1, 0);
    for (int A = 0; A < nat; ++A) {
        atom_chunk0[A] = (int32_t)ch_atom.size();
        for (int64_t e = nl->sph_ptr[A]; e < nl->sph_ptr[A + 1]; e += kChunk) {
            ch_atom.push_back(A);
            ch_beg.push_back((int32_t)e);
            ch_end.push_back((int32_t)std::min<int64_t>(e + kChunk, nl->sph_ptr[A + 1]));
        }
    }
    atom_chunk0[nat] = (int32_t)ch_atom.size();
    nl->nchunks = (int)ch_atom.size();

    // point-centric table: for every point, the (atom, projector values)
    // entries of the spheres holding it, atoms ascending
    std::vector<int32_t> cnt(g->np + 1, 0);
    for (int64_t e = 0; e < nnz; ++e) cnt[nl->sph_idx[e] + 1]++;
    for (int64_t p = 0; p < g->np; ++p) cnt[p + 1] += cnt[p];
    std::vector<int32_t> fillpos(cnt.begin(), cnt.end() - 1);
    std::vector<int32_t> ent_atom(nnz);
    std::vector<double> ent_g(npj * nnz);
    for (int A = 0; A < nat; ++A)
        for (int64_t e = nl->sph_ptr[A]; e < nl->sph_ptr[A + 1]; ++e) {
            const int64_t p = nl->sph_idx[e];
            const int32_t k = fillpos[p]++;
            ent_atom[k] = A;
            for (int i = 0; i < npj; ++i) ent_g[npj * (int64_t)k + i] = nl->gamma[npj * e + i];
        }
    std::vector<int32_t> brick_nl(std::max<int64_t>(g->nbricks, 1), 0);
    if (g->kernels_ok)
        for (int64_t b = 0; b < g->nbricks; ++b) {
            const BrickRec &r = g->bricks_host[b];
            const int64_t n = __builtin_popcountll(r.mask);
            brick_nl[b] = cnt[r.start + n] > cnt[r.start];
        }

    // the points that lie in at least one sphere, ascending
    std::vector<int32_t> nl_pts;
    for (int64_t p = 0; p < g->np; ++p)
        if (cnt[p + 1] > cnt[p]) nl_pts.push_back((int32_t)p);
    nl->nnlpts = (int64_t)nl_pts.size();

    std::vector<int32_t> sph32(nnz);
    for (int64_t e = 0; e < nnz; ++e) sph32[e] = (int32_t)nl->sph_idx[e];
    std::vector<float> g32(nl->gamma.begin(), nl->gamma.end());
    std::vector<float> eg32(ent_g.begin(), ent_g.end());

    nl->host_only = g->host_only;
    if (nl->host_only) {
        *out = nl;
        return RS_OK;
    }
    rs_status st = RS_OK;
    if (!st) st = nl->chunk_atom.upload(ch_atom);
    if (!st) st = nl->chunk_beg.upload(ch_beg);
    if (!st) st = nl->chunk_end.upload(ch_end);
    if (!st) st = nl->atom_chunk0.upload(atom_chunk0);
    if (!st) st = nl->d_sph_idx.upload(sph32);
    if (!st) st = nl->d_gamma64.upload(nl->gamma);
    if (!st) st = nl->d_gamma32.upload(g32);
    if (!st) st = nl->d_D.upload(nl->D);
    if (!st) st = nl->pt_ptr.upload(cnt);
    if (!st) st = nl->ent_atom.upload(ent_atom);
    if (!st) st = nl->ent_gamma64.upload(ent_g);
    if (!st) st = nl->ent_gamma32.upload(eg32);
    if (!st) st = nl->brick_nl.upload(brick_nl);
    if (!st) st = nl->nl_pts.upload(nl_pts);
    if (!st) st = nl->partial.alloc(sizeof(double) * npj * (size_t)max_states * std::max(nl->nchunks, 1));
    if (!st) st = nl->dp.alloc(sizeof(double) * npj * (size_t)max_states * std::max(nat, 1));
    if (st) { delete nl; return st; }
    *out = nl;
    return RS_OK;
}

extern "C" void rs_nl_destroy(rs_nl *nl) { delete nl; }

extern "C" rs_status rs_nl_info(const rs_nl *nl, int64_t *nnz, int32_t *ncolours, int32_t *nproj) {
    if (!nl) return rs::fail(RS_EINVAL, "rs_nl_info: null handle");
    if (nnz) *nnz = (int64_t)nl->sph_idx.size();
    if (ncolours) *ncolours = nl->ncolours;
    if (nproj) *nproj = nl->npj;
    return RS_OK;
}

extern "C" rs_status rs_nl_export(const rs_nl *nl, int64_t *sph_ptr, int64_t *sph_idx,
                                  double *gamma, int32_t *colour) {
    if (!nl) return rs::fail(RS_EINVAL, "rs_nl_export: null handle");
    if (sph_ptr) std::memcpy(sph_ptr, nl->sph_ptr.data(), nl->sph_ptr.size() * sizeof(int64_t));
    if (sph_idx && !nl->sph_idx.empty()) std::memcpy(sph_idx, nl->sph_idx.data(), nl->sph_idx.size() * sizeof(int64_t));
    if (gamma && !nl->gamma.empty()) std::memcpy(gamma, nl->gamma.data(), nl->gamma.size() * sizeof(double));
    if (colour && nl->nat) std::memcpy(colour, nl->colour.data(), nl->colour.size() * sizeof(int32_t));
    return RS_OK;
}
