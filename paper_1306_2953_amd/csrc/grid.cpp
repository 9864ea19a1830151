// Host construction of the grid index map (Sec. 2, Sec. 5.1) and of the
// per-brick tables the stencil kernels read.  Built with -ffp-contract=off:
// membership is integer-only and coordinates are (i - c) * h rounded as
// written.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.hpp"

namespace {

constexpr int kReach = 4;   // stencil half-width (25-point star)

struct SphereRule { int64_t q, Q; };

SphereRule sphere_rule(double radius, double h) {
    const double x = radius / h;
    const double qr = std::nearbyint(x);
    const int64_t q = (int64_t)qr;
    if (std::fabs(x - qr) <= 1e-9 * std::max<double>((double)q, 1.0)) return {q, q * q};
    return {(int64_t)std::floor(x), (int64_t)std::floor(x * x)};
}

}  // namespace

extern "C" rs_status rs_grid_create(const rs_grid_desc *d, rs_grid **out) {
    using namespace rs;
    if (!d || !out) return fail(RS_EINVAL, "rs_grid_create: null argument");
    *out = nullptr;
    if (!(d->h > 0) || !std::isfinite(d->h)) return fail(RS_EINVAL, "grid spacing must be > 0");
    int br[3] = {d->brick[0], d->brick[1], d->brick[2]};
    if (br[0] == 0 && br[1] == 0 && br[2] == 0) br[0] = br[1] = br[2] = 4;
    for (int a = 0; a < 3; ++a)
        if (br[a] < 1 || br[a] > 4096) return fail(RS_EINVAL, "brick edges must be >= 1");

    auto g = new (std::nothrow) rs_grid();
    if (!g) return fail(RS_ENOMEM, "host allocation failed");
    g->kind = d->kind;
    g->h = d->h;
    g->n = d->n;
    g->radius = d->radius;
    g->host_only = (d->flags & RS_GRID_HOST_ONLY) != 0;
    for (int a = 0; a < 3; ++a) g->brick[a] = br[a];

    int64_t lo_in[3] = {0, 0, 0}, ext[3] = {0, 0, 0}, pad = 0, Q = 0;
    if (d->kind == RS_GRID_SPHERE) {
        if (!(d->radius > 0)) { delete g; return fail(RS_EINVAL, "sphere radius must be > 0"); }
        SphereRule r = sphere_rule(d->radius, d->h);
        if (r.q > 20000) { delete g; return fail(RS_EINVAL, "sphere too large"); }
        for (int a = 0; a < 3; ++a) { lo_in[a] = -r.q; ext[a] = 2 * r.q + 1; }
        pad = kReach; Q = r.Q;
        g->centre = 0.0;
    } else if (d->kind == RS_GRID_UNION) {
        if (!(d->radius > 0) || !std::isfinite(d->radius)) { delete g; return fail(RS_EINVAL, "sphere radius must be > 0"); }
        if (d->natoms < 1 || !d->centres) { delete g; return fail(RS_EINVAL, "a union of spheres needs natoms >= 1 centres"); }
        for (int a = 0; a < 3; ++a) {
            double cmin = d->centres[a], cmax = d->centres[a];
            for (int i = 1; i < d->natoms; ++i) {
                const double c = d->centres[3 * i + a];
                if (!std::isfinite(c)) { delete g; return fail(RS_EINVAL, "atom centres must be finite"); }
                cmin = std::min(cmin, c);
                cmax = std::max(cmax, c);
            }
            if (!std::isfinite(cmin) || !std::isfinite(cmax)) { delete g; return fail(RS_EINVAL, "atom centres must be finite"); }
            const double flo = std::floor((cmin - d->radius) / d->h), fhi = std::ceil((cmax + d->radius) / d->h);
            if (!(fhi - flo < 40000.0)) { delete g; return fail(RS_EINVAL, "union of spheres too large"); }
            lo_in[a] = (int64_t)flo;
            ext[a] = (int64_t)fhi - lo_in[a] + 1;
        }
        pad = kReach;
        g->centre = 0.0;
        g->centres.assign(d->centres, d->centres + 3 * (size_t)d->natoms);
    } else if (d->kind == RS_GRID_BOX || d->kind == RS_GRID_PERIODIC) {
        if (d->n < 1 || d->n > 20000) { delete g; return fail(RS_EINVAL, "box edge out of range"); }
        for (int a = 0; a < 3; ++a) { lo_in[a] = 0; ext[a] = d->n; }
        pad = d->kind == RS_GRID_BOX ? kReach : 0;
        g->centre = d->kind == RS_GRID_BOX ? 0.5 * (double)(d->n - 1) : 0.0;
        if (d->kind == RS_GRID_PERIODIC)
            for (int a = 0; a < 3; ++a)
                if (d->n % br[a]) { delete g; return fail(RS_EINVAL, "periodic edge must be a multiple of the brick"); }
    } else {
        delete g;
        return fail(RS_EINVAL, "unknown grid kind");
    }
    for (int a = 0; a < 3; ++a) {
        g->lo[a] = lo_in[a] - pad;
        g->L[a] = ext[a] + 2 * pad;
        g->nb[a] = (g->L[a] + br[a] - 1) / br[a];
    }
    const int64_t L0 = g->L[0], L1 = g->L[1], L2 = g->L[2];
    const int64_t ntot = L0 * L1 * L2;
    std::vector<uint8_t> inside(ntot, 0);
    if (d->kind == RS_GRID_UNION) {
        // each atom marks the lattice points of its sphere: ((x - X)^2 +
        // (y - Y)^2) + (z - Z)^2 <= R^2 with x = i h, rounded as written
        const double h = d->h, r2 = d->radius * d->radius;
        for (int at = 0; at < d->natoms; ++at) {
            const double *c = d->centres + 3 * at;
            int64_t b0[3], b1[3];
            for (int a = 0; a < 3; ++a) {
                b0[a] = std::max<int64_t>(0, (int64_t)std::floor((c[a] - d->radius) / h) - 1 - g->lo[a]);
                b1[a] = std::min<int64_t>(g->L[a] - 1, (int64_t)std::ceil((c[a] + d->radius) / h) + 1 - g->lo[a]);
            }
            for (int64_t k = b0[2]; k <= b1[2]; ++k) {
                const double dz = (double)(k + g->lo[2]) * h - c[2];
                for (int64_t j = b0[1]; j <= b1[1]; ++j) {
                    const double dy = (double)(j + g->lo[1]) * h - c[1];
                    for (int64_t i = b0[0]; i <= b1[0]; ++i) {
                        const double dx = (double)(i + g->lo[0]) * h - c[0];
                        if ((dx * dx + dy * dy) + dz * dz <= r2) inside[(k * L1 + j) * L0 + i] = 1;
                    }
                }
            }
        }
    } else {
        for (int64_t k = 0; k < L2; ++k)
            for (int64_t j = 0; j < L1; ++j)
                for (int64_t i = 0; i < L0; ++i) {
                    const int64_t x = i + g->lo[0], y = j + g->lo[1], z = k + g->lo[2];
                    bool in;
                    if (d->kind == RS_GRID_SPHERE) in = x * x + y * y + z * z <= Q;
                    else in = x >= 0 && x < ext[0] && y >= 0 && y < ext[1] && z >= 0 && z < ext[2];
                    inside[(k * L1 + j) * L0 + i] = in;
                }
    }
    auto is_in = [&](int64_t i, int64_t j, int64_t k) -> bool {
        if (i < 0 || j < 0 || k < 0 || i >= L0 || j >= L1 || k >= L2) return false;
        return inside[(k * L1 + j) * L0 + i];
    };

    g->lookup.assign(ntot, -1);
    const int64_t nbx = g->nb[0], nby = g->nb[1], nbz = g->nb[2];
    g->brick_map.assign(nbx * nby * nbz, -1);
    int64_t nbricks = 0;
    std::vector<int64_t> brick_first;   // first inner index per numbered brick
    // pass 1: inner points in brick order
    for (int64_t bz = 0; bz < nbz; ++bz)
        for (int64_t by = 0; by < nby; ++by)
            for (int64_t bx = 0; bx < nbx; ++bx) {
                const int64_t before = g->np;
                for (int sz = 0; sz < br[2]; ++sz)
                    for (int sy = 0; sy < br[1]; ++sy)
                        for (int sx = 0; sx < br[0]; ++sx) {
                            const int64_t i = bx * br[0] + sx, j = by * br[1] + sy, k = bz * br[2] + sz;
                            if (!is_in(i, j, k)) continue;
                            g->lookup[(k * L1 + j) * L0 + i] = g->np++;
                            g->inner.push_back((int32_t)(i + g->lo[0]));
                            g->inner.push_back((int32_t)(j + g->lo[1]));
                            g->inner.push_back((int32_t)(k + g->lo[2]));
                        }
                if (g->np > before) {
                    g->brick_map[(bz * nby + by) * nbx + bx] = (int32_t)nbricks++;
                    brick_first.push_back(before);
                }
            }
    // pass 2: boundary points (finite systems), same order
    if (d->kind != RS_GRID_PERIODIC) {
        for (int64_t bz = 0; bz < nbz; ++bz)
            for (int64_t by = 0; by < nby; ++by)
                for (int64_t bx = 0; bx < nbx; ++bx)
                    for (int sz = 0; sz < br[2]; ++sz)
                        for (int sy = 0; sy < br[1]; ++sy)
                            for (int sx = 0; sx < br[0]; ++sx) {
                                const int64_t i = bx * br[0] + sx, j = by * br[1] + sy, k = bz * br[2] + sz;
                                if (i >= L0 || j >= L1 || k >= L2 || is_in(i, j, k)) continue;
                                bool hit = false;
                                for (int m = 1; m <= kReach && !hit; ++m)
                                    hit = is_in(i + m, j, k) || is_in(i - m, j, k) ||
                                          is_in(i, j + m, k) || is_in(i, j - m, k) ||
                                          is_in(i, j, k + m) || is_in(i, j, k - m);
                                if (!hit) continue;
                                g->nbnd++;
                                g->boundary.push_back((int32_t)(i + g->lo[0]));
                                g->boundary.push_back((int32_t)(j + g->lo[1]));
                                g->boundary.push_back((int32_t)(k + g->lo[2]));
                            }
    }
    g->nbricks = nbricks;

    // per-brick kernel tables (4x4x4 only)
    g->kernels_ok = br[0] == 4 && br[1] == 4 && br[2] == 4;
    if (g->kernels_ok) {
        if (g->np * 64 >= ((int64_t)1 << 31)) {
            // offsets inside one block are 32-bit in the kernels
            g->kernels_ok = false;
        }
    }
    if (g->kernels_ok) {
        g->bricks_host.resize(nbricks);
        for (int64_t bz = 0; bz < nbz; ++bz)
            for (int64_t by = 0; by < nby; ++by)
                for (int64_t bx = 0; bx < nbx; ++bx) {
                    const int32_t b = g->brick_map[(bz * nby + by) * nbx + bx];
                    if (b < 0) continue;
                    BrickRec &r = g->bricks_host[b];
                    r.mask = 0;
                    r.start = (int32_t)brick_first[b];
                    r.flags = 0;
                    for (int s = 0; s < 64; ++s) {
                        const int64_t i = bx * 4 + (s & 3), j = by * 4 + ((s >> 2) & 3), k = bz * 4 + (s >> 4);
                        if (is_in(i, j, k)) r.mask |= (uint64_t)1 << s;
                    }
                    const int64_t c[3] = {bx, by, bz};
                    for (int a = 0; a < 3; ++a)
                        for (int sgn = 0; sgn < 2; ++sgn) {
                            int64_t cc[3] = {c[0], c[1], c[2]};
                            cc[a] += sgn ? 1 : -1;
                            int32_t nbid = -1;
                            if (d->kind == RS_GRID_PERIODIC) {
                                cc[a] = (cc[a] + g->nb[a]) % g->nb[a];
                                nbid = g->brick_map[(cc[2] * nby + cc[1]) * nbx + cc[0]];
                            } else if (cc[a] >= 0 && cc[a] < g->nb[a]) {
                                nbid = g->brick_map[(cc[2] * nby + cc[1]) * nbx + cc[0]];
                            }
                            r.nbr[a * 2 + sgn] = nbid;
                        }
                }
        for (int64_t b = 0; b < nbricks; ++b) {
            BrickRec &r = g->bricks_host[b];
            bool fast = r.mask == ~0ull;
            for (int f = 0; f < 6 && fast; ++f)
                fast = r.nbr[f] >= 0 && g->bricks_host[r.nbr[f]].mask == ~0ull;
            r.flags = fast ? kBrickFast : 0;
        }
        // execution order: z-pencils of 8 x 8 bricks in x-y, the pencils
        // along a 2-D Z-order (Morton) curve, each pencil from low to high z,
        // a Morton curve inside each z layer of a pencil.  Bricks processed
        // together are then spatially compact and a brick's z neighbours are
        // processed just before and after it, while its neighbours are still
        // in L2.
        auto spread = [](uint64_t v, int stride) {
            uint64_t m = 0;
            for (int bit = 0; bit < 21; ++bit) m |= ((v >> bit) & 1) << (stride * bit);
            return m;
        };
        std::vector<std::pair<uint64_t, int32_t>> key;
        key.reserve(nbricks);
        for (int64_t bz = 0; bz < nbz; ++bz)
            for (int64_t by = 0; by < nby; ++by)
                for (int64_t bx = 0; bx < nbx; ++bx) {
                    const int32_t b = g->brick_map[(bz * nby + by) * nbx + bx];
                    if (b < 0) continue;
                    const uint64_t tile = spread(bx >> 3, 2) | (spread(by >> 3, 2) << 1);
                    const uint64_t inner = spread(bx & 7, 2) | (spread(by & 7, 2) << 1);
                    const uint64_t m = (tile << 40) | ((uint64_t)bz << 8) | inner;
                    key.emplace_back(m, b);
                }
        std::sort(key.begin(), key.end());
        std::vector<int32_t> order;
        order.reserve(nbricks);
        for (int pass = 0; pass < 2; ++pass)
            for (int64_t i = 0; i < nbricks; ++i) {
                const bool fast = (g->bricks_host[key[i].second].flags & kBrickFast) != 0;
                if (fast == (pass == 0)) order.push_back(key[i].second);
            }
        g->nfast = 0;
        for (int64_t b = 0; b < nbricks; ++b) g->nfast += (g->bricks_host[b].flags & kBrickFast) != 0;
        // z-marching chunks: tiles of 2 x 2 bricks; each tile's occupied z
        // range cut at a global grid of kMarchCZ-layer bands, so that the
        // chunks of neighbouring tiles cover the same layers and, run
        // together, share their x-y neighbour rows in L2.  Order: band,
        // then the tiles along a 2-D Morton curve.  Table layers: bz0-1 ..
        // bz0+nz, then one absent layer (the kernel's last prefetches read it).
        const bool per = d->kind == RS_GRID_PERIODIC;
        auto wrap = [](int64_t v, int64_t n) { return ((v % n) + n) % n; };
        std::vector<MarchBrick> mtab;
        std::vector<std::pair<uint64_t, MarchChunk>> mfull, mpart;
        const int64_t ntx = (nbx + 1) / 2, nty = (nby + 1) / 2;
        static const int pdx[12] = {0, 1, 0, 1, -1, -1, 2, 2, 0, 1, 0, 1};
        static const int pdy[12] = {0, 0, 1, 1, 0, 1, 0, 1, -1, -1, 2, 2};

        for (int64_t ty = 0; ty < nty; ++ty)
            for (int64_t tx = 0; tx < ntx; ++tx) {
                int64_t zmin = nbz, zmax = -1;
                for (int64_t bz = 0; bz < nbz; ++bz)
                    for (int o = 0; o < 4; ++o) {
                        const int64_t bx = 2 * tx + pdx[o], by = 2 * ty + pdy[o];
                        if (bx < nbx && by < nby && g->brick_map[(bz * nby + by) * nbx + bx] >= 0) {
                            zmin = std::min(zmin, bz);
                            zmax = std::max(zmax, bz);
                        }
                    }
                if (zmax < 0) continue;
                for (int64_t band = zmin / kMarchCZ; band * kMarchCZ <= zmax; ++band) {
                    const int64_t bz0 = std::max(zmin, band * (int64_t)kMarchCZ);
                    const int nz = (int)(std::min(zmax + 1, (band + 1) * (int64_t)kMarchCZ) - bz0);
                    MarchChunk mc{(int32_t)mtab.size(), nz};
                    bool full = true;
                    for (int l = 0; l < nz + 3; ++l) {
                        const int64_t bz = bz0 - 1 + l;
                        for (int pos = 0; pos < 12; ++pos) {
                            int64_t bx = 2 * tx + pdx[pos], by = 2 * ty + pdy[pos], bzz = bz;
                            // a tile brick is written by this chunk when it is
                            // one of the chunk's layers and inside the lattice
                            const bool owned = pos < 4 && bx < nbx && by < nby && l >= 1 && l <= nz &&
                                               bz >= zmin && bz <= zmax;
                            int32_t id = -1;
                            if (l == nz + 2) {
                                id = -1;
                            } else if (per) {
                                bx = wrap(bx, nbx); by = wrap(by, nby); bzz = wrap(bzz, nbz);
                                id = g->brick_map[(bzz * nby + by) * nbx + bx];
                            } else if (bx >= 0 && bx < nbx && by >= 0 && by < nby && bzz >= 0 && bzz < nbz) {
                                id = g->brick_map[(bzz * nby + by) * nbx + bx];
                            }
                            MarchBrick mb{0, 0, -1};
                            if (id >= 0) {
                                mb.mask = g->bricks_host[id].mask;
                                mb.start = g->bricks_host[id].start;
                                mb.id = owned ? id : -1;
                            }
                            if (l <= nz + 1 && (mb.mask != ~0ull || (pos < 4 && l >= 1 && l <= nz && mb.id < 0)))
                                full = false;
                            mtab.push_back(mb);
                        }
                    }
                    const uint64_t key = ((uint64_t)band << 44) | spread(tx, 2) | (spread(ty, 2) << 1);
                    (full ? mfull : mpart).emplace_back(key, mc);
                }
            }
        std::sort(mfull.begin(), mfull.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
        std::sort(mpart.begin(), mpart.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
        std::vector<MarchChunk> mch;
        for (auto &e : mfull) mch.push_back(e.second);
        for (auto &e : mpart) mch.push_back(e.second);
        g->nmarch = (int64_t)mch.size();
        g->nmarch_full = (int64_t)mfull.size();
        if (!g->host_only) {
            rs_status st = g->bricks.upload(g->bricks_host);
            if (!st) st = g->exec.upload(order);
            if (!st) st = g->march_chunk.upload(mch);
            if (!st) st = g->march_tab.upload(mtab);
            if (st) { delete g; return st; }
        }
    }
    *out = g;
    return RS_OK;
}

extern "C" void rs_grid_destroy(rs_grid *g) { delete g; }

extern "C" rs_status rs_grid_info(const rs_grid *g, int64_t *np, int64_t *nbnd,
                                  int64_t *nbricks, int32_t nb[3], int32_t lo[3]) {
    if (!g) return rs::fail(RS_EINVAL, "rs_grid_info: null grid");
    if (np) *np = g->np;
    if (nbnd) *nbnd = g->nbnd;
    if (nbricks) *nbricks = g->nbricks;
    for (int a = 0; a < 3; ++a) {
        if (nb) nb[a] = (int32_t)g->nb[a];
        if (lo) lo[a] = (int32_t)g->lo[a];
    }
    return RS_OK;
}

extern "C" rs_status rs_grid_export(const rs_grid *g, int32_t *inner, int32_t *boundary,
                                    int32_t *brick_map, double *xyz) {
    if (!g) return rs::fail(RS_EINVAL, "rs_grid_export: null grid");
    if (inner && g->np) std::memcpy(inner, g->inner.data(), g->inner.size() * sizeof(int32_t));
    if (boundary && g->nbnd) std::memcpy(boundary, g->boundary.data(), g->boundary.size() * sizeof(int32_t));
    if (brick_map) std::memcpy(brick_map, g->brick_map.data(), g->brick_map.size() * sizeof(int32_t));
    if (xyz)
        for (int64_t p = 0; p < 3 * g->np; ++p) xyz[p] = ((double)g->inner[p] - g->centre) * g->h;
    return RS_OK;
}
