// Internal declarations shared by the host sources of librsdft.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rsdft.h"

namespace rs {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
rs_status fail(rs_status code, const std::string &msg);
rs_status hip_fail(hipError_t e, const char *what);

#define RS_HIP(call)                                        \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return ::rs::hip_fail(e_, #call); \
    } while (0)

// Device buffer owned by a handle.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    rs_status alloc(size_t n) {
        release();
        if (n == 0) n = 16;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            return fail(RS_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed");
        }
        bytes = n;
        return RS_OK;
    }
    template <typename T>
    rs_status upload(const std::vector<T> &v) {
        rs_status st = alloc(v.size() * sizeof(T));
        if (st) return st;
        if (!v.empty()) RS_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
        return RS_OK;
    }
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

// Per-brick table used by the stencil kernels (4x4x4 bricks, 64 slots;
// slot = (z*4 + y)*4 + x).  `start` is the index of the brick's first inner
// point; the point in slot q is start + popcount(mask & ((1<<q)-1)) when bit
// q of mask is set.  nbr: neighbouring bricks along -x,+x,-y,+y,-z,+z
// (-1 = none, i.e. all zeros).  flags & kBrickFast: the brick and its six
// neighbours all exist and hold 64 points each.
constexpr int32_t kBrickFast = 1;
struct BrickRec {
    uint64_t mask;
    int32_t start;
    int32_t flags;
    int32_t nbr[6];
};
static_assert(sizeof(BrickRec) == 40, "BrickRec layout");

// Work of the z-marching stencil kernel: tiles of 2 x 2 bricks in x-y, each
// tile's column of bricks cut along z into chunks of at most kMarchCZ brick
// layers.  A chunk's table holds, for its layers bz0-1 ..
// bz0+nz+1 (nz + 3 layers, the last one always absent), 12 positions per
// layer: the four tile bricks (position bx + 2 by),
// then the neighbours across the -x side (rows 0, 1), the +x side (rows 0,
// 1), the -y side (columns 0, 1) and the +y side (columns 0, 1).  An absent
// brick has mask 0; id is the brick's number where the chunk owns (writes)
// it, -1 otherwise (neighbours, and periodic images of bricks owned by
// another tile).
constexpr int kMarchCZ = 9;    // 36-layer bands measured within 2 % in time, with 10 % more fetched bytes
struct MarchBrick {
    uint64_t mask;
    int32_t start;
    int32_t id;
};
static_assert(sizeof(MarchBrick) == 16, "MarchBrick layout");
struct MarchChunk {
    int32_t tab;   // first MarchBrick of the chunk's table
    int32_t nz;    // brick layers written
};

}  // namespace rs

struct rs_grid {
    int kind = 0;
    double h = 0;
    int n = 0;
    double radius = 0;
    std::vector<double> centres;     // [natoms][3] sphere centres (union grids)
    int brick[3] = {4, 4, 4};
    int64_t lo[3] = {0, 0, 0};   // integer coordinate of lattice origin
    int64_t L[3] = {0, 0, 0};    // lattice dims
    int64_t nb[3] = {0, 0, 0};   // brick lattice dims
    double centre = 0;           // x = (i - centre) h
    int64_t np = 0, nbnd = 0;
    std::vector<int32_t> inner;      // [np][3]
    std::vector<int32_t> boundary;   // [nbnd][3]
    std::vector<int32_t> brick_map;  // [nb2][nb1][nb0]
    std::vector<int64_t> lookup;     // lattice -> inner index (or -1)
    bool host_only = false;
    // device tables (4x4x4 bricks only)
    bool kernels_ok = false;
    int64_t nbricks = 0;
    std::vector<rs::BrickRec> bricks_host;
    rs::DevBuf bricks;       // BrickRec[nbricks]
    rs::DevBuf exec;         // int32[nbricks]: fast bricks, then the others,
                             // each list in Morton (Z-curve) order
    int64_t nfast = 0;
    // z-marching work: chunks whose 12 x (nz + 2) table entries are all full
    // bricks (and whose tile bricks are owned) first, then the others
    rs::DevBuf march_chunk;  // MarchChunk[nmarch]
    rs::DevBuf march_tab;    // MarchBrick[...]
    int64_t nmarch = 0, nmarch_full = 0;
    int64_t lattice_index(int64_t i, int64_t j, int64_t k) const {
        return ((k - lo[2]) * L[1] + (j - lo[1])) * L[0] + (i - lo[0]);
    }
};

struct rs_nl {
    bool host_only = false;
    int nat = 0;
    int lmax = 1;
    int npj = 4;                    // projectors per atom, (lmax+1)^2
    int max_states = 0;
    double dv = 0;
    std::vector<int64_t> sph_ptr;   // [nat+1]
    std::vector<int64_t> sph_idx;   // [nnz]
    std::vector<double> gamma;      // [nnz][npj]
    std::vector<int32_t> colour;    // [nat]
    std::vector<double> D;          // [nat][npj]
    int ncolours = 0;
    // projection work split: chunks of sphere entries
    int nchunks = 0;
    rs::DevBuf chunk_atom, chunk_beg, chunk_end, atom_chunk0;  // int32
    rs::DevBuf d_sph_idx;                                       // int32 [nnz]
    rs::DevBuf d_gamma64, d_gamma32;                            // [nnz][npj]
    rs::DevBuf d_D;                                             // double [nat][npj]
    // point-centric table for the fused apply
    rs::DevBuf pt_ptr;                                          // int32 [np+1]
    rs::DevBuf ent_atom;                                        // int32 [nent]
    rs::DevBuf ent_gamma64, ent_gamma32;                        // [nent][npj]
    rs::DevBuf brick_nl;                                        // int32 [nbricks]
    rs::DevBuf nl_pts;                                          // int32 [nnlpts]
    int64_t nnlpts = 0;
    // scratch
    rs::DevBuf partial;   // double [max_states][nchunks][npj]
    rs::DevBuf dp;        // dtype  [max_states][nat][npj]  (D * projection)
};
