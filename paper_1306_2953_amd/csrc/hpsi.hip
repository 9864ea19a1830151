// H psi on gfx950 (Sec. 5): finite-difference kinetic stencil, local
// potential and Kleinman-Bylander projectors for blocks of states.
//
// Layout: psi[blk][point][B], the B states of a block contiguous per point
// (Sec. 4), points in brick order (Sec. 5.1).  One lane owns one state of one
// 4x4x4 brick: lanes s = 0..B-1 of a lane group read a contiguous row of B
// values per point, so every load is a coalesced B*sizeof(T) segment.  The
// lane walks the 48 grid lines of its brick (16 per axis); each line needs the
// 4 values of the brick and 4 of each face neighbour brick (the stencil reaches
// 4 points, exactly one brick edge), so a brick's 64 outputs cost 7-9 loads
// per output and no neighbour table (the brick's 64-bit occupancy mask and
// first-point index locate every point).  Points outside the domain are zero
// and cost no memory traffic.
#include "internal.hpp"

namespace rs {
namespace {

// Maps work-group ids so that consecutive bricks land on the same XCD: the
// hardware deals work-groups to the 8 XCDs round-robin.
__device__ __forceinline__ int xcd_remap(int wg, int nwg_pad) {
    return (wg & 7) * (nwg_pad >> 3) + (wg >> 3);
}

// Buffer resources: raw (stride 0) buffers whose loads at offsets beyond
// num_records return zero and whose stores there are dropped.  Points
// outside the domain get such an offset, so no branch guards a load.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
// kOOB plus any lane offset (< 64 KiB) stays above every buffer size the
// launchers accept (kMaxField), so it never wraps into range.
constexpr uint32_t kOOB = 0xFFFF0000u;
constexpr uint64_t kMaxField = 0xFFFE0000ull;

__device__ __forceinline__ rsrc_t make_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename T> __device__ __forceinline__ T bload(rsrc_t r, uint32_t off);
template <> __device__ __forceinline__ float bload<float>(rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <> __device__ __forceinline__ double bload<double>(rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
template <typename T> __device__ __forceinline__ void bstore(T v, rsrc_t r, uint32_t off);
template <> __device__ __forceinline__ void bstore<float>(float v, rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)off, 0, 0);
}
template <> __device__ __forceinline__ void bstore<double>(double v, rsrc_t r, uint32_t off) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 0);
}

// Byte offset of the point in slot q of a brick (mask, start), scaled by
// `row` bytes per point, or kOOB when the slot holds no point.
__device__ __forceinline__ uint32_t slot_off(uint64_t mask, int start, int q, uint32_t row) {
    const uint32_t idx = (uint32_t)(start + __popcll(mask & ((1ull << q) - 1ull)));
    return ((mask >> q) & 1ull) ? idx * row : kOOB;
}

template <typename T, int B>
__device__ __forceinline__ T ld_slot(rsrc_t r, uint64_t mask, int start, int q, uint32_t lane_off) {
    return bload<T>(r, slot_off(mask, start, q, B * sizeof(T)) + lane_off);
}

template <typename T>
__device__ __forceinline__ T line_term(const T *v, int i, T c1, T c2, T c3, T c4) {
    // v[0..]: a line of values with 4 before output i's centre (at v[4+i]).
    const T c0v = v[4 + i];
    T t = c1 * ((v[5 + i] - c0v) + (v[3 + i] - c0v));
    t += c2 * ((v[6 + i] - c0v) + (v[2 + i] - c0v));
    t += c3 * ((v[7 + i] - c0v) + (v[1 + i] - c0v));
    t += c4 * ((v[8 + i] - c0v) + (v[0 + i] - c0v));
    return t;
}

// Hides a value from common-subexpression elimination so that slot offsets
// are recomputed (two integer ops) instead of being kept live in registers.
__device__ __forceinline__ uint64_t opaque(uint64_t m) {
    uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
    asm volatile("" : "+v"(lo), "+v"(hi));
    return ((uint64_t)hi << 32) | lo;
}

// One lane group (B lanes, one state each) computes NZ z-planes (16 points
// each) of one brick, starting at plane Z0; NZ = 4 is the whole brick, NZ = 2
// half of it (used for FP64 to halve the register footprint).  The planes'
// own values stay in registers; every neighbour-brick value is loaded once.
template <typename T, int B, int NZ, int Z0>
__device__ __forceinline__ void
hpsi_brick_body(const BrickRec *__restrict__ bricks, int b, int blk,
                const T *__restrict__ psi, T *__restrict__ hpsi, const T *__restrict__ vloc,
                int64_t blk_stride, T pre, T c1, T c2, T c3, T c4,
                const int32_t *__restrict__ brick_nl, const int32_t *__restrict__ pt_ptr,
                const int32_t *__restrict__ ent_atom, const T *__restrict__ ent_gamma,
                const T *__restrict__ dp, int nat) {
    constexpr int NP = 16 * NZ;             // points per lane group
    constexpr int z0 = Z0;
    const int s = threadIdx.x % B;
    const uint32_t fbytes = (uint32_t)(blk_stride * sizeof(T));
    const rsrc_t rp = make_rsrc(psi + blk * blk_stride, fbytes);
    const rsrc_t rh = make_rsrc(hpsi + blk * blk_stride, fbytes);
    const rsrc_t rv = make_rsrc(vloc, (uint32_t)(blk_stride / B * sizeof(T)));
    const uint32_t lo = s * sizeof(T);

    const BrickRec br = bricks[b];
    uint64_t nm[6];
    int ns[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int j = br.nbr[f];
        nm[f] = j >= 0 ? bricks[j].mask : 0ull;
        ns[f] = j >= 0 ? bricks[j].start : 0;
    }
    const int s0 = br.start;
    uint64_t m0 = br.mask;

    T own[NP], acc[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int q = z0 * 16 + k;
        own[k] = ld_slot<T, B>(rp, m0, s0, q, lo);
        acc[k] = bload<T>(rv, slot_off(m0, s0, q, sizeof(T))) * own[k];
    }
    // x lines
#pragma unroll
    for (int zz = 0; zz < NZ; ++zz)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            T v[12];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                const int q = ((z0 + zz) * 4 + y) * 4 + x;
                v[x] = ld_slot<T, B>(rp, nm[0], ns[0], q, lo);
                v[4 + x] = own[(zz * 4 + y) * 4 + x];
                v[8 + x] = ld_slot<T, B>(rp, nm[1], ns[1], q, lo);
            }
#pragma unroll
            for (int x = 0; x < 4; ++x) acc[(zz * 4 + y) * 4 + x] += pre * line_term(v, x, c1, c2, c3, c4);
            __builtin_amdgcn_sched_barrier(0);
        }
    // y lines
#pragma unroll
    for (int zz = 0; zz < NZ; ++zz)
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            T v[12];
#pragma unroll
            for (int y = 0; y < 4; ++y) {
                const int q = ((z0 + zz) * 4 + y) * 4 + x;
                v[y] = ld_slot<T, B>(rp, nm[2], ns[2], q, lo);
                v[4 + y] = own[(zz * 4 + y) * 4 + x];
                v[8 + y] = ld_slot<T, B>(rp, nm[3], ns[3], q, lo);
            }
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[(zz * 4 + y) * 4 + x] += pre * line_term(v, y, c1, c2, c3, c4);
            __builtin_amdgcn_sched_barrier(0);
        }
    // z lines: a column of NZ + 8 values around the lane group's planes
    m0 = opaque(m0);
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            T v[NZ + 8];
#pragma unroll
            for (int j = 0; j < NZ + 8; ++j) {
                const int z = z0 - 4 + j;       // brick-local z of column entry j
                if (z < 0) {
                    v[j] = ld_slot<T, B>(rp, nm[4], ns[4], ((z + 4) * 4 + y) * 4 + x, lo);
                } else if (z >= 4) {
                    v[j] = ld_slot<T, B>(rp, nm[5], ns[5], ((z - 4) * 4 + y) * 4 + x, lo);
                } else if (z >= z0 && z < z0 + NZ) {
                    v[j] = own[((z - z0) * 4 + y) * 4 + x];
                } else {
                    v[j] = ld_slot<T, B>(rp, m0, s0, (z * 4 + y) * 4 + x, lo);
                }
            }
#pragma unroll
            for (int zz = 0; zz < NZ; ++zz) acc[(zz * 4 + y) * 4 + x] += pre * line_term(v, zz, c1, c2, c3, c4);
            __builtin_amdgcn_sched_barrier(0);
        }
    // non-local part 2, point-centric: sum over the atoms whose sphere holds
    // the point of gamma_A,i(p) * (D_A,i P_A,i,s)
    m0 = opaque(m0);
    if (brick_nl != nullptr && brick_nl[b]) {
        const T *dpb = dp + (int64_t)blk * nat * 4 * B;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int q = z0 * 16 + k;
            if ((m0 >> q) & 1ull) {
                const int p = s0 + __popcll(m0 & ((1ull << q) - 1ull));
                const int k1 = pt_ptr[p + 1];
                for (int e = pt_ptr[p]; e < k1; ++e) {
                    const T *g = ent_gamma + 4 * (int64_t)e;
                    const T *d = dpb + ent_atom[e] * 4 * B + s;
                    acc[k] += g[0] * d[0] + g[1] * d[B] + g[2] * d[2 * B] + g[3] * d[3 * B];
                }
            }
        }
    }
    m0 = opaque(m0);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int q = z0 * 16 + k;
        bstore<T>(acc[k], rh, slot_off(m0, s0, q, B * sizeof(T)) + lo);
    }
}

// Work-group = 4 waves.  With PARTS = 4/NZ lane groups per brick, wave w
// handles part w % PARTS of its bricks, so the part is uniform in a wave.
template <typename T, int B, int NZ>
__global__ void __launch_bounds__(256)
hpsi_brick_kernel(const BrickRec *__restrict__ bricks, int nbricks, int nwg, int nwg_pad,
                  const T *__restrict__ psi, T *__restrict__ hpsi, const T *__restrict__ vloc,
                  int64_t blk_stride, T pre, T c1, T c2, T c3, T c4,
                  const int32_t *__restrict__ brick_nl, const int32_t *__restrict__ pt_ptr,
                  const int32_t *__restrict__ ent_atom, const T *__restrict__ ent_gamma,
                  const T *__restrict__ dp, int nat) {
    constexpr int PARTS = 4 / NZ;
    constexpr int GPW = 64 / B;                 // lane groups per wave
    constexpr int BPWG = 4 * GPW / PARTS;       // bricks per work-group
    const int wg = xcd_remap(blockIdx.x, nwg_pad);
    if (wg >= nwg) return;
    const int wave = threadIdx.x / 64;
    const int part = wave % PARTS;
    const int b = wg * BPWG + (wave / PARTS) * GPW + (threadIdx.x % 64) / B;
    if (b >= nbricks) return;
    if (part == 0)
        hpsi_brick_body<T, B, NZ, 0>(bricks, b, blockIdx.y, psi, hpsi, vloc, blk_stride, pre, c1, c2,
                                     c3, c4, brick_nl, pt_ptr, ent_atom, ent_gamma, dp, nat);
    else if constexpr (PARTS == 2)
        hpsi_brick_body<T, B, NZ, 2>(bricks, b, blockIdx.y, psi, hpsi, vloc, blk_stride, pre, c1, c2,
                                     c3, c4, brick_nl, pt_ptr, ent_atom, ent_gamma, dp, nat);
}

// Non-local part 1 (eq. 6 integrals), stage 1: one work-group per (chunk of
// <= 512 sphere entries of one atom, block).  Lanes: state s, row r; rows
// stride through the chunk; FP64 sums are reduced over rows in a fixed tree.
template <typename T, int B>
__global__ void __launch_bounds__(256)
nl_partial_kernel(const int32_t *__restrict__ chunk_beg, const int32_t *__restrict__ chunk_end,
                  const int32_t *__restrict__ sph_idx, const T *__restrict__ gamma,
                  const T *__restrict__ psi, int64_t blk_stride, double *__restrict__ partial,
                  int nchunks) {
    constexpr int R = 256 / B;
    __shared__ double red[4][256];
    const int chunk = blockIdx.x, blk = blockIdx.y;
    const int s = threadIdx.x % B, r = threadIdx.x / B;
    const int e0 = chunk_beg[chunk], e1 = chunk_end[chunk];
    psi += blk * blk_stride;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (int e = e0 + r; e < e1; e += R) {
        const double x = (double)psi[sph_idx[e] * B + s];
        const T *g = gamma + 4 * (int64_t)e;
        a0 += (double)g[0] * x;
        a1 += (double)g[1] * x;
        a2 += (double)g[2] * x;
        a3 += (double)g[3] * x;
    }
    red[0][threadIdx.x] = a0;
    red[1][threadIdx.x] = a1;
    red[2][threadIdx.x] = a2;
    red[3][threadIdx.x] = a3;
    __syncthreads();
#pragma unroll
    for (int st = R / 2; st > 0; st >>= 1) {
        if (r < st)
#pragma unroll
            for (int i = 0; i < 4; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + st * B];
        __syncthreads();
    }
    if (r == 0)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            partial[(((int64_t)blk * nchunks + chunk) * 4 + i) * B + s] = red[i][s];
}

// Stage 2: sum an atom's chunks in order; P = h^3 sum, DP = D * P.
template <typename T>
__global__ void __launch_bounds__(256)
nl_final_kernel(const int32_t *__restrict__ atom_chunk0, const double *__restrict__ partial,
                const double *__restrict__ D, T *__restrict__ proj, T *__restrict__ dp,
                int nat, int nchunks, int B, int64_t total, double dv) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    const int s = (int)(idx % B);
    const int i = (int)((idx / B) % 4);
    const int A = (int)((idx / (4 * B)) % nat);
    const int64_t blk = idx / (4 * (int64_t)B * nat);
    double sum = 0.0;
    for (int c = atom_chunk0[A]; c < atom_chunk0[A + 1]; ++c)
        sum += partial[((blk * nchunks + c) * 4 + i) * B + s];
    const double P = dv * sum;
    if (proj) proj[idx] = (T)P;
    dp[idx] = (T)(D[A * 4 + i] * P);
}

// Standalone non-local part 2 (rs_apply_nl): hpsi += sum gamma D proj, one
// lane per (point, state) of points that lie in at least one sphere.
template <typename T>
__global__ void __launch_bounds__(256)
nl_apply_kernel(const int32_t *__restrict__ pt_ptr, const int32_t *__restrict__ ent_atom,
                const T *__restrict__ ent_gamma, const double *__restrict__ D,
                const T *__restrict__ proj, T *__restrict__ hpsi, int64_t np, int B, int nat) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int blk = blockIdx.y;
    if (idx >= np * B) return;
    const int64_t p = idx / B;
    const int s = (int)(idx % B);
    const int k0 = pt_ptr[p], k1 = pt_ptr[p + 1];
    if (k0 == k1) return;
    const T *pb = proj + (int64_t)blk * nat * 4 * B;
    T acc = T(0);
    for (int k = k0; k < k1; ++k) {
        const int A = ent_atom[k];
        const T *g = ent_gamma + 4 * (int64_t)k;
        const T *pa = pb + A * 4 * B + s;
#pragma unroll
        for (int i = 0; i < 4; ++i) acc += g[i] * (T)D[A * 4 + i] * pa[i * B];
    }
    T *y = hpsi + (int64_t)blk * np * B + idx;
    *y = *y + acc;
}

bool pow2_block(int B) { return B >= 1 && B <= 64 && (B & (B - 1)) == 0; }

template <typename T>
rs_status launch_project(const rs_grid *g, const rs_nl *nl, const T *psi, T *proj, int nblk,
                         int B, hipStream_t st) {
    if (nl->nchunks == 0) return RS_OK;
    const T *gam = sizeof(T) == 8 ? (const T *)nl->d_gamma64.p : (const T *)nl->d_gamma32.p;
    const int64_t stride = g->np * B;
    dim3 grid1(nl->nchunks, nblk);
#define RS_PARTIAL(BB)                                                                      \
    case BB:                                                                                \
        hipLaunchKernelGGL((nl_partial_kernel<T, BB>), grid1, dim3(256), 0, st,            \
                           nl->chunk_beg.as<int32_t>(), nl->chunk_end.as<int32_t>(),       \
                           nl->d_sph_idx.as<int32_t>(), gam, psi, stride,                  \
                           nl->partial.as<double>(), nl->nchunks);                         \
        break;
    switch (B) {
        RS_PARTIAL(1) RS_PARTIAL(2) RS_PARTIAL(4) RS_PARTIAL(8) RS_PARTIAL(16) RS_PARTIAL(32) RS_PARTIAL(64)
    }
#undef RS_PARTIAL
    RS_HIP(hipGetLastError());
    const int64_t total = (int64_t)nblk * nl->nat * 4 * B;
    hipLaunchKernelGGL((nl_final_kernel<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       nl->atom_chunk0.as<int32_t>(), nl->partial.as<double>(), nl->d_D.as<double>(),
                       proj, (T *)nl->dp.p, nl->nat, nl->nchunks, B, total, nl->dv);
    RS_HIP(hipGetLastError());
    return RS_OK;
}

template <typename T>
rs_status launch_hpsi(const rs_grid *g, const rs_nl *nl, const T *vloc, const T *psi, T *hpsi,
                      int nblk, int B, hipStream_t st) {
    if (g->nbricks == 0) return RS_OK;
    if ((uint64_t)g->np * B * sizeof(T) > kMaxField)
        return fail(RS_ENOTSUP, "rs_hpsi_block: one block of fields exceeds 4 GiB");
    const bool with_nl = nl != nullptr && nl->nat > 0;
    if (with_nl) {
        rs_status s = launch_project<T>(g, nl, psi, nullptr, nblk, B, st);
        if (s) return s;
    }
    const double c[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
    const T pre = (T)(-0.5 / (g->h * g->h));
    constexpr int NZ = sizeof(T) == 8 ? 2 : 4;
    const int bpwg = 4 * (64 / B) / (4 / NZ);
    const int nwg = (int)((g->nbricks + bpwg - 1) / bpwg);
    const int nwg_pad = (nwg + 7) & ~7;
    dim3 grid(nwg_pad, nblk);
    const int64_t stride = g->np * B;
    const int32_t *bnl = with_nl ? nl->brick_nl.as<int32_t>() : nullptr;
    const int32_t *ptp = with_nl ? nl->pt_ptr.as<int32_t>() : nullptr;
    const int32_t *eat = with_nl ? nl->ent_atom.as<int32_t>() : nullptr;
    const T *egm = with_nl ? (sizeof(T) == 8 ? (const T *)nl->ent_gamma64.p : (const T *)nl->ent_gamma32.p) : nullptr;
    const T *dp = with_nl ? (const T *)nl->dp.p : nullptr;
    const int nat = with_nl ? nl->nat : 0;
#define RS_HPSI(BB)                                                                          \
    case BB:                                                                                 \
        hipLaunchKernelGGL((hpsi_brick_kernel<T, BB, NZ>), grid, dim3(256), 0, st,              \
                           g->bricks.as<BrickRec>(), (int)g->nbricks, nwg, nwg_pad, psi,    \
                           hpsi, vloc, stride, pre, (T)c[1], (T)c[2], (T)c[3], (T)c[4],      \
                           bnl, ptp, eat, egm, dp, nat);                                     \
        break;
    switch (B) {
        RS_HPSI(1) RS_HPSI(2) RS_HPSI(4) RS_HPSI(8) RS_HPSI(16) RS_HPSI(32) RS_HPSI(64)
    }
#undef RS_HPSI
    RS_HIP(hipGetLastError());
    return RS_OK;
}

rs_status check_fields(const rs_grid *g, const rs_nl *nl, int nblk, int B, int dtype,
                       const char *who) {
    if (!g) return fail(RS_EINVAL, std::string(who) + ": null grid");
    if (g->host_only || (nl && nl->host_only))
        return fail(RS_EINVAL, std::string(who) + ": grid or projector set was built host-only");
    if (!g->kernels_ok) return fail(RS_ENOTSUP, std::string(who) + ": kernels need 4x4x4 bricks");
    if (!pow2_block(B)) return fail(RS_EINVAL, std::string(who) + ": B must be a power of two in [1, 64]");
    if (nblk < 1) return fail(RS_EINVAL, std::string(who) + ": nblk must be >= 1");
    if (nblk > 65535) return fail(RS_EINVAL, std::string(who) + ": nblk too large");
    if (dtype != RS_F64 && dtype != RS_F32) return fail(RS_EINVAL, std::string(who) + ": bad dtype");
    if (nl && (int64_t)nblk * B > nl->max_states)
        return fail(RS_EINVAL, std::string(who) + ": nblk*B exceeds max_states of the projector set");
    return RS_OK;
}

}  // namespace
}  // namespace rs

using namespace rs;

extern "C" rs_status rs_hpsi_block(const rs_grid *g, const rs_nl *nl, const void *vloc,
                                   const void *psi, void *hpsi, int32_t nblk, int32_t B,
                                   int32_t dtype, void *stream) {
    rs_status st = check_fields(g, nl, nblk, B, dtype, "rs_hpsi_block");
    if (st) return st;
    if (!vloc || !psi || !hpsi) return fail(RS_EINVAL, "rs_hpsi_block: null field pointer");
    if (psi == hpsi) return fail(RS_EINVAL, "rs_hpsi_block: psi and hpsi must not alias");
    hipStream_t s = (hipStream_t)stream;
    if (dtype == RS_F64)
        return launch_hpsi<double>(g, nl, (const double *)vloc, (const double *)psi, (double *)hpsi, nblk, B, s);
    return launch_hpsi<float>(g, nl, (const float *)vloc, (const float *)psi, (float *)hpsi, nblk, B, s);
}

extern "C" rs_status rs_project_nl(const rs_grid *g, const rs_nl *nl, const void *psi, void *proj,
                                   int32_t nblk, int32_t B, int32_t dtype, void *stream) {
    rs_status st = check_fields(g, nl, nblk, B, dtype, "rs_project_nl");
    if (st) return st;
    if (!nl || !psi || !proj) return fail(RS_EINVAL, "rs_project_nl: null argument");
    hipStream_t s = (hipStream_t)stream;
    if (dtype == RS_F64)
        return launch_project<double>(g, nl, (const double *)psi, (double *)proj, nblk, B, s);
    return launch_project<float>(g, nl, (const float *)psi, (float *)proj, nblk, B, s);
}

extern "C" rs_status rs_apply_nl(const rs_grid *g, const rs_nl *nl, const void *proj, void *hpsi,
                                 int32_t nblk, int32_t B, int32_t dtype, void *stream) {
    rs_status st = check_fields(g, nl, nblk, B, dtype, "rs_apply_nl");
    if (st) return st;
    if (!nl || !proj || !hpsi) return fail(RS_EINVAL, "rs_apply_nl: null argument");
    if (nl->nat == 0) return RS_OK;
    hipStream_t s = (hipStream_t)stream;
    dim3 grid((unsigned)((g->np * B + 255) / 256), nblk);
    if (dtype == RS_F64)
        hipLaunchKernelGGL((nl_apply_kernel<double>), grid, dim3(256), 0, s, nl->pt_ptr.as<int32_t>(),
                           nl->ent_atom.as<int32_t>(), (const double *)nl->ent_gamma64.p,
                           nl->d_D.as<double>(), (const double *)proj, (double *)hpsi, g->np, B, nl->nat);
    else
        hipLaunchKernelGGL((nl_apply_kernel<float>), grid, dim3(256), 0, s, nl->pt_ptr.as<int32_t>(),
                           nl->ent_atom.as<int32_t>(), (const float *)nl->ent_gamma32.p,
                           nl->d_D.as<double>(), (const float *)proj, (float *)hpsi, g->np, B, nl->nat);
    RS_HIP(hipGetLastError());
    return RS_OK;
}
