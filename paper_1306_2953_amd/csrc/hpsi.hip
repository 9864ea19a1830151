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
//
// FP64 uses a second design, hpsi_march_kernel below: work-groups march
// through 8 x 8-point columns in z with a register window along z and the
// x-y neighbours staged in LDS, which cuts the row reads per output from
// 9-13 to about 3.
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
// Cache policy of the field stores: non-temporal (the outputs are not read
// again by this kernel, so they should not evict neighbour data from L2).
constexpr int kStoreAux = 2;
template <typename T> __device__ __forceinline__ void bstore(T v, rsrc_t r, uint32_t off);
template <> __device__ __forceinline__ void bstore<float>(float v, rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)off, 0, kStoreAux);
}
template <> __device__ __forceinline__ void bstore<double>(double v, rsrc_t r, uint32_t off) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, kStoreAux);
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

// Weights of the stencil written on first differences d_k = v_{k+1} - v_k:
// sum_m c_m (v_{i+m} + v_{i-m} - 2 v_i) = sum_j W_j (d_{i+j} - d_{i-1-j}),
// W_j = sum_{m>j} c_m.  Differences of neighbouring values are exact or
// nearly so, so the cancellation of the plain form (c_0 = -2 sum c_m) never
// happens in FP32, and a line of n values costs n-1 subtractions shared by
// its outputs plus 8 operations per output.
struct StencilW { double w0, w1, w2, w3; };

// R = 1 keeps only the nearest-neighbour term (the 7-point filter); the
// values more than one step away are then never read.
template <typename T, int N, int R>
__device__ __forceinline__ void line_lap(const T (&v)[N], T (&lap)[N - 8], T w0, T w1, T w2, T w3) {
    T d[N - 1];
#pragma unroll
    for (int k = 0; k < N - 1; ++k)
        if (R == 4 || (k >= 3 && k <= N - 5)) d[k] = v[k + 1] - v[k];
#pragma unroll
    for (int i = 0; i < N - 8; ++i) {
        const int p = 4 + i;
        T t = w0 * (d[p] - d[p - 1]);
        if constexpr (R == 4) {
            t += w1 * (d[p + 1] - d[p - 2]);
            t += w2 * (d[p + 2] - d[p - 3]);
            t += w3 * (d[p + 3] - d[p - 4]);
        }
        lap[i] = t;
    }
}

// Uniform buffer loads with the slot offset in a scalar register and the
// lane offset (plus a compile-time immediate) in a vector register.
template <typename T> __device__ __forceinline__ T bload_s(rsrc_t r, uint32_t voff, uint32_t soff);
template <> __device__ __forceinline__ float bload_s<float>(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <> __device__ __forceinline__ double bload_s<double>(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}

// Locates slot q of a brick.  FAST: the brick is full, so slot q is point
// start + q; the byte offset splits into a scalar base per group of K slots
// and an immediate (q mod K) * ROW that fits the instruction's 12-bit offset
// field.  Otherwise the offsets come from a table in LDS that the wave fills
// first; empty slots hold kOOB and the lane offset is added with unsigned
// saturation, so their loads return 0 and their stores are dropped.
template <typename T, int ROW, bool FAST>
struct Slots {
    static constexpr int K = (4096 / ROW) >= 64 ? 64 : (4096 / ROW);
    int start;
    uint32_t base;            // FAST: start * ROW
    const uint32_t *tbl;      // !FAST: 64 byte offsets in LDS
    __device__ __forceinline__ T load(rsrc_t r, uint32_t lane_off, int q) const {
        if constexpr (FAST)
            return bload_s<T>(r, lane_off + (uint32_t)((q % K) * ROW), base + (uint32_t)((q / K) * K * ROW));
        else
            return bload<T>(r, __builtin_elementwise_add_sat(lane_off, tbl[q]));
    }
    __device__ __forceinline__ void store(T v, rsrc_t r, uint32_t lane_off, int q) const {
        if constexpr (FAST) {
            if constexpr (sizeof(T) == 4)
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r,
                                                      (int)(lane_off + (q % K) * ROW), (int)(base + (q / K) * K * ROW),
                                                      kStoreAux);
            else {
                typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r,
                                                      (int)(lane_off + (q % K) * ROW), (int)(base + (q / K) * K * ROW),
                                                      kStoreAux);
            }
        } else {
            bstore<T>(v, r, __builtin_elementwise_add_sat(lane_off, tbl[q]));
        }
    }
    __device__ __forceinline__ bool has(int q) const {
        if constexpr (FAST) return true;
        else return tbl[q] != kOOB;
    }
    // point index of an occupied slot q
    __device__ __forceinline__ int point(int q) const {
        if constexpr (FAST) return start + q;
        else return (int)(tbl[q] / ROW);
    }
};

// Phase fence: the accumulators are materialised (an empty asm that
// reads and writes them) and the scheduler may not move instructions
// across.  Without it the compiler defers all arithmetic to the end and
// issues every load of the brick first, which needs several hundred
// registers and leaves one wave per SIMD; with it each phase's loads are
// consumed before the next phase's are issued.
template <typename T, int N>
__device__ __forceinline__ void phase_fence(T (&acc)[N]) {
#pragma unroll
    for (int k = 0; k < N; ++k) asm volatile("" : "+v"(acc[k]));
    __builtin_amdgcn_sched_barrier(0);
}
#define RS_PHASE() phase_fence(acc)
constexpr int kPhaseLines = 4;     // stencil lines per phase

// One wave computes NZ z-planes (from plane Z0) of one brick for 64 state
// columns: lane l is state (c mod B) of block (c / B), c = 64*colgroup + l.
// Everything that locates points (brick records, masks, offsets) is uniform
// in the wave and lives in scalar registers; a lane's address is its column
// offset plus the uniform slot offset.
template <typename T, int ROW, int NZ, int Z0, bool FAST, int R>
__device__ __forceinline__ void
hpsi_wave(const BrickRec &br, const BrickRec *__restrict__ bricks, int b, rsrc_t rp, rsrc_t rh,
          uint32_t lane_off, const uint32_t *tbl, const T *__restrict__ vloc, T vconst, T pre, T w0,
          T w1, T w2, T w3, const int32_t *__restrict__ brick_nl, const int32_t *__restrict__ pt_ptr,
          const int32_t *__restrict__ ent_atom, const T *__restrict__ ent_gamma,
          const T *__restrict__ dpl, int B) {
    constexpr int NP = 16 * NZ;
    Slots<T, ROW, FAST> nb[6], me;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int j = br.nbr[f];
        nb[f].start = j >= 0 ? bricks[j].start : 0;
        nb[f].base = (uint32_t)nb[f].start * ROW;
        nb[f].tbl = tbl + (f + 1) * 64;
    }
    me.start = br.start;
    me.base = (uint32_t)br.start * ROW;
    me.tbl = tbl;

    T own[NP], acc[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        own[k] = me.load(rp, lane_off, Z0 * 16 + k);
    }
    // x lines
#pragma unroll
    for (int zz = 0; zz < NZ; ++zz)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            T v[12], lap[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                const int q = ((Z0 + zz) * 4 + y) * 4 + x;
                v[x] = (R == 4 || x == 3) ? nb[0].load(rp, lane_off, q) : T(0);
                v[4 + x] = own[(zz * 4 + y) * 4 + x];
                v[8 + x] = (R == 4 || x == 0) ? nb[1].load(rp, lane_off, q) : T(0);
            }
            line_lap<T, 12, R>(v, lap, w0, w1, w2, w3);
#pragma unroll
            for (int x = 0; x < 4; ++x) acc[(zz * 4 + y) * 4 + x] = lap[x];
            if ((zz * 4 + y) % kPhaseLines == kPhaseLines - 1) RS_PHASE();
        }
    // y lines
#pragma unroll
    for (int zz = 0; zz < NZ; ++zz)
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            T v[12], lap[4];
#pragma unroll
            for (int y = 0; y < 4; ++y) {
                const int q = ((Z0 + zz) * 4 + y) * 4 + x;
                v[y] = (R == 4 || y == 3) ? nb[2].load(rp, lane_off, q) : T(0);
                v[4 + y] = own[(zz * 4 + y) * 4 + x];
                v[8 + y] = (R == 4 || y == 0) ? nb[3].load(rp, lane_off, q) : T(0);
            }
            line_lap<T, 12, R>(v, lap, w0, w1, w2, w3);
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[(zz * 4 + y) * 4 + x] += lap[y];
            if ((zz * 4 + x) % kPhaseLines == kPhaseLines - 1) RS_PHASE();
        }
    // z lines: NZ + 8 values around this wave's planes
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            T v[NZ + 8], lap[NZ];
#pragma unroll
            for (int j = 0; j < NZ + 8; ++j) {
                const int z = Z0 - 4 + j;
                if (R == 1 && (j < 3 || j > NZ + 4)) v[j] = T(0);
                else if (z < 0) v[j] = nb[4].load(rp, lane_off, ((z + 4) * 4 + y) * 4 + x);
                else if (z >= 4) v[j] = nb[5].load(rp, lane_off, ((z - 4) * 4 + y) * 4 + x);
                else if (z >= Z0 && z < Z0 + NZ) v[j] = own[((z - Z0) * 4 + y) * 4 + x];
                else v[j] = me.load(rp, lane_off, (z * 4 + y) * 4 + x);
            }
            line_lap<T, NZ + 8, R>(v, lap, w0, w1, w2, w3);
#pragma unroll
            for (int zz = 0; zz < NZ; ++zz) acc[(zz * 4 + y) * 4 + x] += lap[zz];
            if ((y * 4 + x) % kPhaseLines == kPhaseLines - 1) RS_PHASE();
        }
    // local potential (or a constant when vloc is null)
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int q = Z0 * 16 + k;
        const T vp = vloc == nullptr ? vconst : (me.has(q) ? vloc[me.point(q)] : T(0));
        acc[k] = pre * acc[k] + vp * own[k];
    }
    // non-local part 2 for the s and p set (4 projectors per atom; other
    // projector counts are added by nl_add_kernel), point-centric: sum over
    // the atoms whose sphere holds the point of gamma_A,i(p) * (D_A,i P_A,i,s)
    if (brick_nl != nullptr && brick_nl[b]) {
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int q = Z0 * 16 + k;
            if (me.has(q)) {
                const int p = me.point(q);
                const int e1 = pt_ptr[p + 1];
                for (int e = pt_ptr[p]; e < e1; ++e) {
                    const T *g = ent_gamma + 4 * (int64_t)e;
                    const T *d = dpl + ent_atom[e] * 4 * B;
                    acc[k] += g[0] * d[0] + g[1] * d[B] + g[2] * d[2 * B] + g[3] * d[3 * B];
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        me.store(acc[k], rh, lane_off, Z0 * 16 + k);
    }
}

// Work-group = 4 waves.  blockIdx.y selects a group of 64 state columns;
// blockIdx.x (XCD-remapped) a run of bricks from `exec` (one of two lists:
// interior bricks, FAST, whose neighbours are all full, and the rest).  A
// brick is split into 4/NZ parts of NZ z-planes, one wave each.  B is a
// template parameter so that the row size B * sizeof(T) is a constant.
template <typename T, int B, int NZ, bool FAST, int R>
__global__ void __launch_bounds__(256)
hpsi_brick_kernel(const BrickRec *__restrict__ bricks, const int32_t *__restrict__ exec,
                  int nexec, int nwg, int nwg_pad, const T *__restrict__ psi,
                  T *__restrict__ hpsi, const T *__restrict__ vloc, T vconst, int64_t np, int nblk,
                  T pre, T w0, T w1, T w2, T w3,
                  const int32_t *__restrict__ brick_nl, const int32_t *__restrict__ pt_ptr,
                  const int32_t *__restrict__ ent_atom, const T *__restrict__ ent_gamma,
                  const T *__restrict__ dp, int nat) {
    constexpr int PARTS = 4 / NZ;
    constexpr int ROW = B * (int)sizeof(T);
    __shared__ uint32_t tbl_all[FAST ? 1 : 4 * 7 * 64];
    const int wg = xcd_remap(blockIdx.x, nwg_pad);
    if (wg >= nwg) return;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int slot = (wg * 4 + wave) / PARTS;
    const int part = (wg * 4 + wave) % PARTS;
    const int lane = threadIdx.x & 63;
    const uint32_t *tbl = nullptr;
    if constexpr (!FAST) {
        // slot byte offsets of this brick and its six neighbours, one lane
        // per slot: rank of the slot among the occupied ones, or kOOB
        uint32_t *t = tbl_all + wave * 7 * 64;
        const int bb = slot < nexec ? exec[slot] : -1;
#pragma unroll
        for (int f = 0; f < 7; ++f) {
            const int j = bb < 0 ? -1 : (f == 0 ? bb : bricks[bb].nbr[f - 1]);
            uint32_t off = kOOB;
            if (j >= 0) {
                const uint64_t m = bricks[j].mask;
                if ((m >> lane) & 1ull)
                    off = (uint32_t)(bricks[j].start + __popcll(m & ((1ull << lane) - 1ull))) * ROW;
            }
            t[f * 64 + lane] = off;
        }
        __syncthreads();
        tbl = t;
    }
    if (slot >= nexec) return;
    const int b = exec[slot];
    const int col = blockIdx.y * 64 + lane;
    const int blk0 = (blockIdx.y * 64) / B;          // first block of this column group
    const int blk = col / B;
    if (blk >= nblk) return;
    const int s = col % B;
    const int nb_here = min(nblk - blk0, 64 / B);
    const int64_t blk_elems = np * B;
    const uint32_t bytes = (uint32_t)(nb_here * blk_elems * sizeof(T));
    const rsrc_t rp = make_rsrc(psi + blk0 * blk_elems, bytes);
    const rsrc_t rh = make_rsrc(hpsi + blk0 * blk_elems, bytes);
    const uint32_t lane_off = (uint32_t)(((blk - blk0) * blk_elems + s) * sizeof(T));
    const T *dpl = dp ? dp + (int64_t)blk * nat * 4 * B + s : nullptr;
    const BrickRec br = bricks[b];
#define RS_PART(ZZ)                                                                            \
    hpsi_wave<T, ROW, NZ, ZZ, FAST, R>(br, bricks, b, rp, rh, lane_off, tbl, vloc, vconst, pre, w0, w1, w2, w3, \
                                    brick_nl, pt_ptr, ent_atom, ent_gamma, dpl, B)
    if (part == 0) RS_PART(0);
    if constexpr (PARTS >= 2) { if (part == 1) RS_PART(NZ); }
    if constexpr (PARTS == 4) { if (part == 2) RS_PART(2 * NZ); if (part == 3) RS_PART(3 * NZ); }
#undef RS_PART
}

// ---------------------------------------------------------------------------
// z-marching kernel (the 25-point stencil of Sec. 5.1 plus the local
// potential; the projector term is added by nl_add_kernel).  A work-group
// owns one chunk: a column of 2 x 2 bricks (8 x 8 points in x-y) over nz
// brick layers, for one group of SG = 16 state columns (128 bytes of each
// point row).  It walks the chunk plane by plane in z:
//  - each thread owns one point of one state column and keeps the values of
//    planes z-4 .. z+7 of that point in registers, so the z part of the
//    stencil costs one load per output, issued three planes ahead;
//  - the plane's 8 x 8 points and their x/y neighbours (4 deep on each side,
//    128 points) are staged in LDS as a 16 x 16-point plane of 128-byte rows;
//    the neighbour rows are fetched two planes ahead as 16-byte pieces.  Two
//    LDS planes alternate, so one barrier per plane suffices.
// A chunk reads its own rows once, the 4 planes below and above it, and
// each plane's 128 x-y neighbour points, which the chunks of neighbouring
// tiles in the same band (run at the same time on the same XCD) have just
// brought into L2.  The step is unrolled over the 12 slots of the register
// window, so every ring index is a compile-time constant and no load sits
// under a branch; a chunk's last 4 or 8 planes run the first steps of the
// same body.
constexpr int kMW = 12;   // register window planes

// Measured choices: 128-byte state groups (64-byte groups fit two
// work-groups per CU but ran slower), one point per thread (1024 threads, 4
// waves per SIMD; 2 or 4 points per thread need 182-256 VGPRs), the plain
// form c0 v + sum c_m (v_-m + v_+m) (no cancellation concern in FP64).  FP32
// fields run on the per-brick kernel above: a 2- or 4-point FP32 variant of
// this kernel in the first-difference form measured 714 / 549 us per H psi
// of 128 states on the 904k-point sphere against the per-brick 456 us.
constexpr int kMarchSG = 16;              // FP64 state columns per work-group
template <int B, bool FULL>
__global__ void __launch_bounds__(64 * kMarchSG)
hpsi_march_kernel(const MarchChunk *__restrict__ chunks, const MarchBrick *__restrict__ tab, int nchunk,
                  int nsg, int nwg_pad, const double *__restrict__ psi, double *__restrict__ hpsi,
                  const double *__restrict__ vloc, double vconst, int64_t np, double pre, double w0, double w1,
                  double w2, double w3) {
    typedef double T;
    constexpr int SG = kMarchSG;
    constexpr int NT = 64 * SG;
    constexpr int RB = SG * (int)sizeof(T);
    constexpr int ROWB = B * (int)sizeof(T);
    constexpr int NPC = RB / 16;                 // 16-byte pieces of a point row
    constexpr int KH = 128 * NPC / NT;           // neighbour pieces per thread and plane
    constexpr int PLANE = 256 * RB;
    constexpr int PH = 2;                        // planes of neighbour prefetch
    static_assert(RB == 128 && KH == 1 && 12 % PH == 0, "launch shape");
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    __shared__ __attribute__((aligned(16))) unsigned char lds[2 * PLANE];
    __shared__ MarchBrick ltab[(kMarchCZ + 3) * 12];

    // work item: chunk wg % nchunk of state group wg / nchunk; each XCD runs
    // a contiguous run of the chunk list (bands of z, tiles in Morton order),
    // so the tiles it holds at once are neighbours at the same depth
    const int wg = xcd_remap(blockIdx.x, nwg_pad);
    if (wg >= nchunk * nsg) return;
    const MarchChunk ch = chunks[wg % nchunk];
    const int sg = wg / nchunk;
    const int tid = threadIdx.x;
    for (int i = tid; i < (ch.nz + 3) * 12; i += NT) ltab[i] = tab[ch.tab + i];
    __syncthreads();

    // thread: state column s of the group, point (x0, y0) of the tile
    const int s = tid % SG, pg = tid / SG;
    const int x0 = pg % 8, y0 = pg / 8;
    const int opos = (x0 >> 2) + 2 * (y0 >> 2);
    const int oq = (y0 & 3) * 4 + (x0 & 3);
    const int blk = sg * SG / B, s0 = sg * SG % B;
    const int64_t bel = np * B;
    const rsrc_t rp = make_rsrc(psi + blk * bel, (uint32_t)(bel * sizeof(T)));
    const rsrc_t rh = make_rsrc(hpsi + blk * bel, (uint32_t)(bel * sizeof(T)));
    // without vloc every potential load reads past a zero-sized buffer (0)
    const rsrc_t rv = make_rsrc(vloc, vloc ? (uint32_t)(np * sizeof(T)) : 0u);
    const uint32_t loff = (uint32_t)((s0 + s) * sizeof(T));
    const uint32_t hc = (uint32_t)(s0 * sizeof(T) + (tid % NPC) * 16);

    // neighbour pieces: point hp of the 128 (32 rows of 4 points: 16 x-side
    // rows, then 16 y-side rows), 16-byte piece tid % NPC of its row
    int hpos[KH], hq[KH];
    uint32_t hlds[KH];
#pragma unroll
    for (int k = 0; k < KH; ++k) {
        const int hp = (tid + k * NT) / NPC;
        const int hr = hp >> 2, xi = hp & 3;
        int X, Y;
        if (hr < 16) {
            const int side = hr >> 3, y = hr & 7;
            hpos[k] = 4 + 2 * side + (y >> 2);
            hq[k] = (y & 3) * 4 + xi;
            X = side ? 12 + xi : xi;
            Y = y + 4;
        } else {
            const int r = hr - 16, side = r >> 3, yv = (r & 7) >> 1, xb = r & 1;
            hpos[k] = 8 + 2 * side + xb;
            hq[k] = yv * 4 + xi;
            X = 4 + 4 * xb + xi;
            Y = side ? 12 + yv : yv;
        }
        hlds[k] = (uint32_t)((Y * 16 + X) * RB + (tid % NPC) * 16);
    }

    // point index of slot q of a table entry, or -1
    auto prow = [&](const MarchBrick &mb, int q) -> int {
        if constexpr (FULL) {
            return mb.start + q;
        } else {
            const uint64_t m = mb.mask;
            return ((m >> q) & 1ull) ? mb.start + __popcll(m & ((1ull << q) - 1ull)) : -1;
        }
    };
    // byte offset of point r's row plus extra (full chunks: r is never -1)
    auto roff = [&](int r, uint32_t extra, uint32_t rowb) -> uint32_t {
        if constexpr (FULL) return (uint32_t)r * rowb + extra;
        else return r < 0 ? kOOB : (uint32_t)r * rowb + extra;
    };
    // the thread's point in plane p
    auto load_own = [&](int p, T &w) {
        const MarchBrick mb = ltab[(p >> 2) * 12 + opos];
        w = bload<T>(rp, roff(prow(mb, (p & 3) * 16 + oq), loff, ROWB));
    };
    auto load_halo = [&](int p, u32x4 (&h)[KH]) {
#pragma unroll
        for (int k = 0; k < KH; ++k) {
            const MarchBrick mb = ltab[(p >> 2) * 12 + hpos[k]];
            h[k] = __builtin_amdgcn_raw_buffer_load_b128(rp, (int)roff(prow(mb, (p & 3) * 16 + hq[k]), hc, ROWB), 0, 0);
        }
    };
    auto load_v = [&](int p, T &v) {
        const MarchBrick mb = ltab[(p >> 2) * 12 + opos];
        v = bload<T>(rv, roff(prow(mb, (p & 3) * 16 + oq), 0u, (uint32_t)sizeof(T)));
    };

    T win[kMW];
    u32x4 hreg[PH][KH];
    T vreg[3];
    const int zend = 4 + 4 * ch.nz;            // output planes [4, zend) of the chunk's numbering

    // prologue: window planes 0 .. 10, neighbours of planes 4 .. 3 + PH, V
    // of planes 4 and 5
#pragma unroll
    for (int p = 0; p < 11; ++p) load_own(p, win[p]);
#pragma unroll
    for (int p = 4; p < 4 + PH; ++p) load_halo(p, hreg[p % PH]);
    load_v(4, vreg[4 % 3]);
    load_v(5, vreg[5 % 3]);

    // one plane z = zb + K (zb = 4 mod 12)
    auto step = [&](int zb, auto KC) {
        constexpr int K = decltype(KC)::value;
        const int z = zb + K;
        // keep the steps apart: interleaving two planes' arithmetic costs
        // registers (and occupancy)
        __builtin_amdgcn_sched_barrier(0);
        constexpr int c0 = (4 + K) % kMW;                 // window slot of plane z
        constexpr int hs = (4 + K) % PH;                  // neighbour ring slot of plane z
        constexpr int vs = (4 + K) % 3;                   // V ring slot of plane z
        unsigned char *pl = lds + (K & 1) * PLANE;
        // stage plane z: own values from the window, neighbours from the ring
        *(T *)(pl + ((y0 + 4) * 16 + x0 + 4) * RB + s * sizeof(T)) = win[c0];
#pragma unroll
        for (int k = 0; k < KH; ++k) *(u32x4 *)(pl + hlds[k]) = hreg[hs][k];
        // prefetch: window plane z + 7, neighbours of plane z + PH, V of z + 2
        load_own(z + 7, win[(c0 + 7) % kMW]);
        load_halo(z + PH, hreg[hs]);
        load_v(z + 2, vreg[(vs + 2) % 3]);
        __syncthreads();
        const MarchBrick mb = ltab[(z >> 2) * 12 + opos];
        if constexpr (!FULL) {
            // a wave holds one 4-point x row of one brick: when none of its
            // points exists in this plane there is nothing to compute or
            // store (its zeros are already staged for the neighbours)
            if (((mb.mask >> ((z & 3) * 16 + (y0 & 3) * 4)) & 0xFull) == 0) return;
        }
        const unsigned char *L = pl + (y0 * 16 + x0) * RB + s * sizeof(T);   // point (x0 - 4, y0 - 4)
        auto at = [&](int dx, int dy) -> T { return *(const T *)(L + ((dy + 4) * 16 + dx + 4) * RB); };
        // c0 v + sum_m c_m (v_-m + v_+m) per axis, c_m = W_(m-1) - W_m
        // (W_4 = 0) and c0 = -2 W_0
        const T c1 = w0 - w1, c2 = w1 - w2, c3 = w2 - w3, c4 = w3, c0x3 = T(-6) * w0;
        const T cc[5] = {T(0), c1, c2, c3, c4};
        T sum = c0x3 * win[c0];
#pragma unroll
        for (int m = 1; m <= 4; ++m) {
            sum += cc[m] * (at(-m, 0) + at(m, 0));
            sum += cc[m] * (at(0, -m) + at(0, m));
            sum += cc[m] * (win[(c0 + kMW - m) % kMW] + win[(c0 + m) % kMW]);
        }
        const T acc = pre * sum + (vreg[vs] + vconst) * win[c0];
        if (FULL || mb.id >= 0) bstore<T>(acc, rh, roff(prow(mb, (z & 3) * 16 + oq), loff, ROWB));
    };
    int zb = 4;
    for (; zb + kMW <= zend; zb += kMW) {
        step(zb, std::integral_constant<int, 0>{});
        step(zb, std::integral_constant<int, 1>{});
        step(zb, std::integral_constant<int, 2>{});
        step(zb, std::integral_constant<int, 3>{});
        step(zb, std::integral_constant<int, 4>{});
        step(zb, std::integral_constant<int, 5>{});
        step(zb, std::integral_constant<int, 6>{});
        step(zb, std::integral_constant<int, 7>{});
        step(zb, std::integral_constant<int, 8>{});
        step(zb, std::integral_constant<int, 9>{});
        step(zb, std::integral_constant<int, 10>{});
        step(zb, std::integral_constant<int, 11>{});
    }
    // a last group of 4 or 8 planes: the first steps of the same body
    if (zb < zend) {
        step(zb, std::integral_constant<int, 0>{});
        step(zb, std::integral_constant<int, 1>{});
        step(zb, std::integral_constant<int, 2>{});
        step(zb, std::integral_constant<int, 3>{});
        if (zb + 4 < zend) {
            step(zb, std::integral_constant<int, 4>{});
            step(zb, std::integral_constant<int, 5>{});
            step(zb, std::integral_constant<int, 6>{});
            step(zb, std::integral_constant<int, 7>{});
        }
    }
}

// Projector term added to an H psi computed without it: hpsi += sum over the
// spheres holding the point of gamma_A,i(p) (D_A,i P_A,i), i < NPJ, one lane
// per (state, point) of the points that lie in a sphere (eq. 6).  A lane
// serves up to 4 blocks: the entry loads are shared and the 4 updates are
// independent; the H psi values are read before the entries, so their
// latency overlaps the entry loads.  nnl * B < 2^32 (checked by the host).
template <typename T, int NPJ>
__global__ void __launch_bounds__(256)
nl_add_kernel(const int32_t *__restrict__ nl_pts, int64_t nnl, const int32_t *__restrict__ pt_ptr,
              const int32_t *__restrict__ ent_atom, const T *__restrict__ ent_gamma, const T *__restrict__ dp,
              T *__restrict__ hpsi, int64_t np, int B, int nat, int nblk) {
    const uint32_t idx = blockIdx.x * 256u + threadIdx.x;
    if ((int64_t)idx >= nnl * B) return;
    const int blk0 = 4 * blockIdx.y;
    const int nb = min(4, nblk - blk0);
    const int p = nl_pts[idx / (uint32_t)B];
    const int s = (int)(idx % (uint32_t)B);
    const int64_t dstride = (int64_t)nat * NPJ * B;
    const T *dpl = dp + blk0 * dstride + s;
    T acc[4] = {T(0), T(0), T(0), T(0)}, y[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (k < nb) y[k] = hpsi[((int64_t)(blk0 + k) * np + p) * B + s];
    for (int e = pt_ptr[p], e1 = pt_ptr[p + 1]; e < e1; ++e) {
        T g[NPJ];
#pragma unroll
        for (int i = 0; i < NPJ; ++i) g[i] = ent_gamma[NPJ * (int64_t)e + i];
        const T *d = dpl + ent_atom[e] * NPJ * B;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < nb) {
                const T *dk = d + k * dstride;
                T t = g[0] * dk[0];
#pragma unroll
                for (int i = 1; i < NPJ; ++i) t += g[i] * dk[i * B];
                acc[k] += t;
            }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (k < nb) hpsi[((int64_t)(blk0 + k) * np + p) * B + s] = y[k] + acc[k];
}

// Non-local part 1 (eq. 6 integrals), stage 1: one work-group per (chunk of
// <= 512 sphere entries of one atom, block).  Lanes: state s, row r; rows
// stride through the chunk; FP64 sums are reduced over rows in a fixed tree.
template <typename T, int B, int NPJ>
__global__ void __launch_bounds__(256)
nl_partial_kernel(const int32_t *__restrict__ chunk_beg, const int32_t *__restrict__ chunk_end,
                  const int32_t *__restrict__ sph_idx, const T *__restrict__ gamma,
                  const T *__restrict__ psi, int64_t blk_stride, double *__restrict__ partial,
                  int nchunks) {
    constexpr int R = 256 / B;
    __shared__ double red[NPJ][256];
    const int chunk = blockIdx.x, blk = blockIdx.y;
    const int s = threadIdx.x % B, r = threadIdx.x / B;
    const int e0 = chunk_beg[chunk], e1 = chunk_end[chunk];
    psi += blk * blk_stride;
    double a[NPJ];
#pragma unroll
    for (int i = 0; i < NPJ; ++i) a[i] = 0.0;
    // unrolled so that several entries' gathers are in flight per thread
#pragma unroll 4
    for (int e = e0 + r; e < e1; e += R) {
        const double x = (double)psi[sph_idx[e] * B + s];
        const T *g = gamma + NPJ * (int64_t)e;
#pragma unroll
        for (int i = 0; i < NPJ; ++i) a[i] += (double)g[i] * x;
    }
#pragma unroll
    for (int i = 0; i < NPJ; ++i) red[i][threadIdx.x] = a[i];
    __syncthreads();
#pragma unroll
    for (int st = R / 2; st > 0; st >>= 1) {
        if (r < st)
#pragma unroll
            for (int i = 0; i < NPJ; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + st * B];
        __syncthreads();
    }
    if (r == 0)
#pragma unroll
        for (int i = 0; i < NPJ; ++i)
            partial[(((int64_t)blk * nchunks + chunk) * NPJ + i) * B + s] = red[i][s];
}

// Stage 2: sum an atom's chunks in order; P = h^3 sum, DP = D * P.
template <typename T>
__global__ void __launch_bounds__(256)
nl_final_kernel(const int32_t *__restrict__ atom_chunk0, const double *__restrict__ partial,
                const double *__restrict__ D, T *__restrict__ proj, T *__restrict__ dp,
                int nat, int npj, int nchunks, int B, int64_t total, double dv) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    const int s = (int)(idx % B);
    const int i = (int)((idx / B) % npj);
    const int A = (int)((idx / (npj * B)) % nat);
    const int64_t blk = idx / (npj * (int64_t)B * nat);
    double sum = 0.0;
    for (int c = atom_chunk0[A]; c < atom_chunk0[A + 1]; ++c)
        sum += partial[((blk * nchunks + c) * npj + i) * B + s];
    const double P = dv * sum;
    if (proj) proj[idx] = (T)P;
    dp[idx] = (T)(D[A * npj + i] * P);
}

// Standalone non-local part 2 (rs_apply_nl): hpsi += sum gamma D proj, one
// lane per (point, state) of points that lie in at least one sphere.
template <typename T>
__global__ void __launch_bounds__(256)
nl_apply_kernel(const int32_t *__restrict__ pt_ptr, const int32_t *__restrict__ ent_atom,
                const T *__restrict__ ent_gamma, const double *__restrict__ D,
                const T *__restrict__ proj, T *__restrict__ hpsi, int64_t np, int B, int nat, int npj) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int blk = blockIdx.y;
    if (idx >= np * B) return;
    const int64_t p = idx / B;
    const int s = (int)(idx % B);
    const int k0 = pt_ptr[p], k1 = pt_ptr[p + 1];
    if (k0 == k1) return;
    const T *pb = proj + (int64_t)blk * nat * npj * B;
    T acc = T(0);
    for (int k = k0; k < k1; ++k) {
        const int A = ent_atom[k];
        const T *g = ent_gamma + npj * (int64_t)k;
        const T *pa = pb + A * npj * B + s;
        for (int i = 0; i < npj; ++i) acc += g[i] * (T)D[A * npj + i] * pa[i * B];
    }
    T *y = hpsi + (int64_t)blk * np * B + idx;
    *y = *y + acc;
}

// z planes per wave of the per-brick kernel on interior bricks (FP64, FP32)
// and on the others
constexpr int kNZF64 = 1, kNZF32 = 2, kNZS64 = 1, kNZS32 = 2;

bool pow2_block(int B) { return B >= 1 && B <= 64 && (B & (B - 1)) == 0; }

template <typename T>
rs_status launch_project(const rs_grid *g, const rs_nl *nl, const T *psi, T *proj, int nblk,
                         int B, hipStream_t st) {
    if (nl->nchunks == 0) return RS_OK;
    const T *gam = sizeof(T) == 8 ? (const T *)nl->d_gamma64.p : (const T *)nl->d_gamma32.p;
    const int64_t stride = g->np * B;
    dim3 grid1(nl->nchunks, nblk);
    auto partial = [&](auto npj_c) {
        constexpr int NPJ = decltype(npj_c)::value;
#define RS_PARTIAL(BB)                                                                      \
    case BB:                                                                                \
        hipLaunchKernelGGL((nl_partial_kernel<T, BB, NPJ>), grid1, dim3(256), 0, st,       \
                           nl->chunk_beg.as<int32_t>(), nl->chunk_end.as<int32_t>(),       \
                           nl->d_sph_idx.as<int32_t>(), gam, psi, stride,                  \
                           nl->partial.as<double>(), nl->nchunks);                         \
        break;
        switch (B) {
            RS_PARTIAL(1) RS_PARTIAL(2) RS_PARTIAL(4) RS_PARTIAL(8) RS_PARTIAL(16) RS_PARTIAL(32) RS_PARTIAL(64)
        }
#undef RS_PARTIAL
    };
    switch (nl->npj) {
        case 1: partial(std::integral_constant<int, 1>{}); break;
        case 4: partial(std::integral_constant<int, 4>{}); break;
        case 9: partial(std::integral_constant<int, 9>{}); break;
        case 16: partial(std::integral_constant<int, 16>{}); break;
        default: return fail(RS_EINVAL, "project: unsupported projector count");
    }
    RS_HIP(hipGetLastError());
    const int64_t total = (int64_t)nblk * nl->nat * nl->npj * B;
    hipLaunchKernelGGL((nl_final_kernel<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       nl->atom_chunk0.as<int32_t>(), nl->partial.as<double>(), nl->d_D.as<double>(),
                       proj, (T *)nl->dp.p, nl->nat, nl->npj, nl->nchunks, B, total, nl->dv);
    RS_HIP(hipGetLastError());
    return RS_OK;
}

// The projector term added to a finished H psi (nl_add_kernel), for the
// set's projector count; the projections must be in nl->dp.
template <typename T>
rs_status launch_nl_add(const rs_grid *g, const rs_nl *nl, T *hpsi, int nblk, int B, hipStream_t st) {
    if (nl->nnlpts == 0) return RS_OK;
    if ((int64_t)nl->nnlpts * B > (int64_t)UINT32_MAX - 255)
        return fail(RS_EINVAL, "stencil: too many projector points x states for one launch");
    const T *egm = sizeof(T) == 8 ? (const T *)nl->ent_gamma64.p : (const T *)nl->ent_gamma32.p;
    dim3 gn((unsigned)((nl->nnlpts * B + 255) / 256), (nblk + 3) / 4);
#define RS_NLADD(NPJ)                                                                                   \
    case NPJ:                                                                                           \
        hipLaunchKernelGGL((nl_add_kernel<T, NPJ>), gn, dim3(256), 0, st, nl->nl_pts.as<int32_t>(),     \
                           nl->nnlpts, nl->pt_ptr.as<int32_t>(), nl->ent_atom.as<int32_t>(), egm,       \
                           (const T *)nl->dp.p, hpsi, g->np, B, nl->nat, nblk);                         \
        break;
    switch (nl->npj) {
        RS_NLADD(1) RS_NLADD(4) RS_NLADD(9) RS_NLADD(16)
        default: return fail(RS_EINVAL, "stencil: unsupported projector count");
    }
#undef RS_NLADD
    RS_HIP(hipGetLastError());
    return RS_OK;
}

// Applies out = pre * L psi + V psi (+ V_nl psi when nl is given), L the
// star stencil with first-difference weights w0..w3 (see line_lap); V is
// vloc, or the constant vconst when vloc is null.  R = 1: nearest
// neighbours only (w1 = w2 = w3 = 0).
template <typename T, int R = 4>
rs_status launch_stencil(const rs_grid *g, const rs_nl *nl, const T *vloc, T vconst, const T *psi, T *hpsi,
                         int nblk, int B, double pre_d, const double w[4], hipStream_t st) {
    if (g->nbricks == 0) return RS_OK;
    if ((uint64_t)g->np * 64 * sizeof(T) > kMaxField)
        return fail(RS_ENOTSUP, "stencil: 64 state columns of the grid exceed 4 GiB");
    const bool with_nl = nl != nullptr && nl->nat > 0;
    if (with_nl) {
        rs_status s = launch_project<T>(g, nl, psi, nullptr, nblk, B, st);
        if (s) return s;
    }
    const T pre = (T)pre_d;
    const int ncg = (nblk * B + 63) / 64;
    const int32_t *bnl = with_nl ? nl->brick_nl.as<int32_t>() : nullptr;
    const int32_t *ptp = with_nl ? nl->pt_ptr.as<int32_t>() : nullptr;
    const int32_t *eat = with_nl ? nl->ent_atom.as<int32_t>() : nullptr;
    const T *egm = with_nl ? (sizeof(T) == 8 ? (const T *)nl->ent_gamma64.p : (const T *)nl->ent_gamma32.p) : nullptr;
    const T *dp = with_nl ? (const T *)nl->dp.p : nullptr;
    const int nat = with_nl ? nl->nat : 0;
    const int npj = with_nl ? nl->npj : 0;
    const T w0 = (T)w[0], w1 = (T)w[1], w2 = (T)w[2], w3 = (T)w[3];
    // z-marching kernel (FP64): the full stencil when the block splits into
    // state groups of 16 columns (B = 16, 32, 64)
    if constexpr (R == 4 && sizeof(T) == 8) {
        constexpr int SG = kMarchSG;
        constexpr int NT = 64 * SG;
        const int64_t nsg = (int64_t)nblk * B / SG;
        if (g->nmarch > 0 && B % SG == 0 && g->nmarch * nsg < (1ll << 30)) {
            for (int pass = 0; pass < 2; ++pass) {
                const bool full = pass == 0;
                const int64_t n = full ? g->nmarch_full : g->nmarch - g->nmarch_full;
                if (n == 0) continue;
                const MarchChunk *mc = g->march_chunk.as<MarchChunk>() + (full ? 0 : g->nmarch_full);
                const int nwg_pad = (int)((n * nsg + 7) & ~7ll);
                dim3 grid(nwg_pad);
#define RS_MARCH_LAUNCH(BB)                                                                          \
    case BB:                                                                                         \
        if constexpr (BB % SG == 0) {                                                                \
            if (full)                                                                                \
                hipLaunchKernelGGL((hpsi_march_kernel<BB, true>), grid, dim3(NT), 0, st, mc,         \
                                   g->march_tab.as<MarchBrick>(), (int)n, (int)nsg, nwg_pad, psi, hpsi, vloc, vconst, \
                                   g->np, pre, w0, w1, w2, w3);                                      \
            else                                                                                     \
                hipLaunchKernelGGL((hpsi_march_kernel<BB, false>), grid, dim3(NT), 0, st, mc,        \
                                   g->march_tab.as<MarchBrick>(), (int)n, (int)nsg, nwg_pad, psi, hpsi, vloc, vconst, \
                                   g->np, pre, w0, w1, w2, w3);                                      \
        }                                                                                            \
        break;
                switch (B) {
                    RS_MARCH_LAUNCH(8) RS_MARCH_LAUNCH(16) RS_MARCH_LAUNCH(32) RS_MARCH_LAUNCH(64)
                    default:
                        return fail(RS_ENOTSUP, "stencil: no z-marching kernel for this block size");
                }
#undef RS_MARCH_LAUNCH
                RS_HIP(hipGetLastError());
            }
            return with_nl ? launch_nl_add<T>(g, nl, hpsi, nblk, B, st) : RS_OK;
        }
    }
    // interior bricks: NZF planes per wave; surface bricks: NZS.  The s and
    // p projector term is fused into the brick kernel; other projector
    // counts are added afterwards
    const bool fuse_nl = with_nl && npj == 4;
    if (!fuse_nl) bnl = nullptr;
    constexpr int NZF = sizeof(T) == 8 ? kNZF64 : kNZF32;
    constexpr int NZS = sizeof(T) == 8 ? kNZS64 : kNZS32;
    for (int pass = 0; pass < 2; ++pass) {
        const bool fast = pass == 0;
        const int64_t nexec = fast ? g->nfast : g->nbricks - g->nfast;
        if (nexec == 0) continue;
        const int32_t *ex = g->exec.as<int32_t>() + (fast ? 0 : g->nfast);
        const int parts = 4 / (fast ? NZF : NZS);
        const int nwg = (int)((nexec * parts + 3) / 4);
        const int nwg_pad = (nwg + 7) & ~7;
        dim3 grid(nwg_pad, ncg);
#define RS_HPSI(BB)                                                                                \
    case BB:                                                                                       \
        if (fast)                                                                                  \
            hipLaunchKernelGGL((hpsi_brick_kernel<T, BB, NZF, true, R>), grid, dim3(256), 0, st,     \
                               g->bricks.as<BrickRec>(), ex, (int)nexec, nwg, nwg_pad, psi, hpsi, \
                               vloc, vconst, g->np, nblk, pre, w0, w1, w2, w3, bnl, ptp, eat, egm, \
                               dp, nat);                                                          \
        else                                                                                       \
            hipLaunchKernelGGL((hpsi_brick_kernel<T, BB, NZS, false, R>), grid, dim3(256), 0, st,    \
                               g->bricks.as<BrickRec>(), ex, (int)nexec, nwg, nwg_pad, psi, hpsi, \
                               vloc, vconst, g->np, nblk, pre, w0, w1, w2, w3, bnl, ptp, eat, egm, \
                               dp, nat);                                                          \
        break;
        switch (B) {
            RS_HPSI(1) RS_HPSI(2) RS_HPSI(4) RS_HPSI(8) RS_HPSI(16) RS_HPSI(32) RS_HPSI(64)
        }
#undef RS_HPSI
        RS_HIP(hipGetLastError());
    }
    return with_nl && !fuse_nl ? launch_nl_add<T>(g, nl, hpsi, nblk, B, st) : RS_OK;
}

// The 25-point kinetic stencil of Sec. 5.1: c = (8/5, -1/5, 8/315, -1/560),
// W_j = sum_{m>j} c_m, prefactor -1/(2h^2).
template <typename T>
rs_status launch_hpsi(const rs_grid *g, const rs_nl *nl, const T *vloc, const T *psi, T *hpsi,
                      int nblk, int B, hipStream_t st) {
    const double c1 = 8.0 / 5.0, c2 = -1.0 / 5.0, c3 = 8.0 / 315.0, c4 = -1.0 / 560.0;
    const double w[4] = {c1 + c2 + c3 + c4, c2 + c3 + c4, c3 + c4, c4};
    return launch_stencil<T>(g, nl, vloc, T(0), psi, hpsi, nblk, B, -0.5 / (g->h * g->h), w, st);
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

// Complex states under a real operator: a block of B complex states is the
// block of 2B real columns (re, im interleaved) in the same memory; the
// real dtype and column count replace the complex ones.
rs_status real_columns(int32_t &dtype, int32_t &B, const char *who) {
    if (dtype != RS_C128 && dtype != RS_C64) return RS_OK;
    if (B > 32) return fail(RS_EINVAL, std::string(who) + ": complex blocks hold at most 32 states");
    dtype = dtype == RS_C128 ? RS_F64 : RS_F32;
    B *= 2;
    return RS_OK;
}

}  // namespace
}  // namespace rs

using namespace rs;

extern "C" rs_status rs_hpsi_block(const rs_grid *g, const rs_nl *nl, const void *vloc,
                                   const void *psi, void *hpsi, int32_t nblk, int32_t B,
                                   int32_t dtype, void *stream) {
    rs_status st = real_columns(dtype, B, "rs_hpsi_block");
    if (st) return st;
    st = check_fields(g, nl, nblk, B, dtype, "rs_hpsi_block");
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
    rs_status st = real_columns(dtype, B, "rs_project_nl");
    if (st) return st;
    st = check_fields(g, nl, nblk, B, dtype, "rs_project_nl");
    if (st) return st;
    if (!nl || !psi || !proj) return fail(RS_EINVAL, "rs_project_nl: null argument");
    hipStream_t s = (hipStream_t)stream;
    if (dtype == RS_F64)
        return launch_project<double>(g, nl, (const double *)psi, (double *)proj, nblk, B, s);
    return launch_project<float>(g, nl, (const float *)psi, (float *)proj, nblk, B, s);
}

extern "C" rs_status rs_apply_nl(const rs_grid *g, const rs_nl *nl, const void *proj, void *hpsi,
                                 int32_t nblk, int32_t B, int32_t dtype, void *stream) {
    rs_status st = real_columns(dtype, B, "rs_apply_nl");
    if (st) return st;
    st = check_fields(g, nl, nblk, B, dtype, "rs_apply_nl");
    if (st) return st;
    if (!nl || !proj || !hpsi) return fail(RS_EINVAL, "rs_apply_nl: null argument");
    if (nl->nat == 0) return RS_OK;
    hipStream_t s = (hipStream_t)stream;
    dim3 grid((unsigned)((g->np * B + 255) / 256), nblk);
    if (dtype == RS_F64)
        hipLaunchKernelGGL((nl_apply_kernel<double>), grid, dim3(256), 0, s, nl->pt_ptr.as<int32_t>(),
                           nl->ent_atom.as<int32_t>(), (const double *)nl->ent_gamma64.p,
                           nl->d_D.as<double>(), (const double *)proj, (double *)hpsi, g->np, B, nl->nat, nl->npj);
    else
        hipLaunchKernelGGL((nl_apply_kernel<float>), grid, dim3(256), 0, s, nl->pt_ptr.as<int32_t>(),
                           nl->ent_atom.as<int32_t>(), (const float *)nl->ent_gamma32.p,
                           nl->d_D.as<double>(), (const float *)proj, (float *)hpsi, g->np, B, nl->nat, nl->npj);
    RS_HIP(hipGetLastError());
    return RS_OK;
}

namespace rs {

rs_status hpsi_apply(const rs_grid *g, const rs_nl *nl, const void *vloc, const void *psi, void *hpsi,
                     int nblk, int B, int dtype, hipStream_t st) {
    if (dtype == RS_F64)
        return launch_hpsi<double>(g, nl, (const double *)vloc, (const double *)psi, (double *)hpsi, nblk, B, st);
    return launch_hpsi<float>(g, nl, (const float *)vloc, (const float *)psi, (float *)hpsi, nblk, B, st);
}

// Filter preconditioner: K r = alpha r + (1 - alpha)/6 (sum of the six nearest
// neighbours) = r + (1 - alpha)/6 L7 r, L7 the 7-point second difference
// (first-difference weights (1, 0, 0, 0)); zero outside the domain.
rs_status filter_apply(const rs_grid *g, double alpha, const void *r, void *out, int nblk, int B, int dtype,
                       hipStream_t st) {
    const double w[4] = {1.0, 0.0, 0.0, 0.0};
    const double pre = (1.0 - alpha) / 6.0;
    if (dtype == RS_F64)
        return launch_stencil<double, 1>(g, nullptr, nullptr, 1.0, (const double *)r, (double *)out, nblk, B, pre, w,
                                         st);
    return launch_stencil<float, 1>(g, nullptr, nullptr, 1.0f, (const float *)r, (float *)out, nblk, B, pre, w, st);
}

}  // namespace rs

namespace rs {

// Kinetic energy alone: out = T psi (the 25-point stencil, no potential).
rs_status kinetic_apply(const rs_grid *g, const void *psi, void *out, int nblk, int B, int dtype,
                        hipStream_t st) {
    const double c1 = 8.0 / 5.0, c2 = -1.0 / 5.0, c3 = 8.0 / 315.0, c4 = -1.0 / 560.0;
    const double w[4] = {c1 + c2 + c3 + c4, c2 + c3 + c4, c3 + c4, c4};
    const double pre = -0.5 / (g->h * g->h);
    if (dtype == RS_F64)
        return launch_stencil<double>(g, nullptr, nullptr, 0.0, (const double *)psi, (double *)out, nblk, B, pre, w,
                                      st);
    return launch_stencil<float>(g, nullptr, nullptr, 0.0f, (const float *)psi, (float *)out, nblk, B, pre, w, st);
}

}  // namespace rs
