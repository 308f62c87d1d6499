// D3Q7 reactive-diffusion lattice Boltzmann kernels for CDNA4 (gfx950).
//
// Scheme: Chen et al., arXiv 1410.1914, Section 4, Eq. (21) with g_eq = w_i C
// (Eq. 23 read on D3Q7), C = sum_i g_i (Eq. 24), sink S = -k n C (Eqs. 17b, 18a);
// boundaries of Section 3.5 (Eqs. 19, 20a, 20b).
//
// Layout (one wave64 = one 64-voxel row segment = one 64-bit mask word):
//   * Fluid voxels are stored compactly in x-fastest order; the compact index of a
//     fluid lane is pre + mbcnt(m) (the number of fluid lanes below it).
//   * A segment record (SegRec) carries the masks and compact prefixes of the four
//     neighbour rows, so the compact index of the +-y / +-z neighbour is the same
//     mbcnt on that row's mask: no per-voxel neighbour table exists.
//   * Populations are blocked by 64 compact voxels: f[(j / 64) * 448 + i * 64 + j % 64],
//     i = rest, +x, -x, +y, -y, +z, -z, so one block (1792 bytes) holds the seven
//     populations of 64 consecutive fluid voxels and a wave's own loads and stores
//     stay inside one or two DRAM pages.  They are stored post-collision as
//     g_i = f_i - w_i c_sh(x), c_sh the linear empty-box profile (a constant for the
//     reactive problem).  The shift is exact; it keeps the stored
//     values small so FP32 storage resolves the fluxes.
//   * Arithmetic is FP64: the seven FP32 loads are summed exactly, and each stored
//     value carries a single rounding, so rounding does not bias the mass balance.
//   * Populations are read and written through buffer resources: 32-bit byte
//     offsets, and the hardware range check turns any out-of-range access into a
//     zero read or a dropped write.
//
// Every stored value is read exactly once per step (by the voxel it streams into,
// or by its own voxel when bounced back), and every fluid voxel writes its seven
// populations once: 56 bytes per fluid update, plus the relaxation rate in Knudsen
// problems and the segment record (120 bytes per 64 voxels).
#include "kernels.h"

namespace cl {
namespace {

// dword 3 of a raw (untyped, unswizzled) buffer resource on the gfx9 family
constexpr int kRawBuffer = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, kRawBuffer);
}

// the b32 buffer builtins move raw 32-bit words: reinterpret, never convert
__device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

__device__ __forceinline__ void st(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, 0);
}

__device__ __forceinline__ int mbcnt64(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int bit(uint64_t m, int lane) { return (int)((m >> lane) & 1ull); }

// Per-lane select by the lane's bit of a wave-uniform mask held in an SGPR pair:
// one v_cndmask_b32 instead of a 64-bit shift, an and and a compare.
__device__ __forceinline__ uint32_t lane_sel(uint64_t m, uint32_t if_set, uint32_t if_clear) {
    uint32_t r;
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(r) : "v"(if_clear), "v"(if_set), "s"(m));
    return r;
}

// Workgroups are dealt to the 8 XCDs round robin; renumber them so that each XCD
// works on one contiguous eighth of the list (neighbour rows then share its L2).
__device__ __forceinline__ int logical_block(int b, int nblk, int remap) {
    if (!remap || nblk < 8) return b;
    const int q = nblk >> 3, r = nblk & 7;
    const int x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

// The same renumbering with each XCD walking its eighth backwards.  Steps
// alternate between the two, so a step starts on the segments the previous step
// touched last: their lines are still in that XCD's L2 and in the last-level cache.
__device__ __forceinline__ int logical_block_reversed(int b, int nblk, int remap) {
    if (!remap || nblk < 8) return nblk - 1 - b;
    const int q = nblk >> 3, r = nblk & 7;
    const int x = b & 7, len = q + (x < r ? 1 : 0);
    return x * q + min(x, r) + (len - 1 - (b >> 3));
}

// x of a lane of a segment (lanes from brk on lie on the next row)
__device__ __forceinline__ int lane_x(const SegRec &R, int lane) {
    return lane < (int)R.brk ? (int)R.x0 + lane : lane - (int)R.brk;
}

// catalyst face-neighbour count of reacting lanes, from the record's bit planes
__device__ __forceinline__ int react_n(const SegRec &R, int lane) {
    return bit(R.n0, lane) + 2 * bit(R.n1, lane) + 4 * bit(R.n2, lane);
}

// Element and byte offsets of population i of compact voxel j in the blocked layout.
__device__ __forceinline__ int64_t pidx(int i, int64_t j) { return (j >> 6) * 448 + i * 64 + (j & 63); }
__device__ __forceinline__ uint32_t pbyte(uint32_t j) { return 4u * (448u * (j >> 6) + (j & 63u)); }

// Byte offset past every buffer: a lane with nothing to do loads 0 from here.
constexpr uint32_t kOutOfRange = 0xFFFFFFF0u;

// Gather phase of one segment: the seven pulled populations (bounce-back reads the
// voxel's own opposite one) and the relaxation rate, issued without waiting.
template <bool KNUDSEN>
__device__ __forceinline__ void gather(const SegRec &R, __amdgpu_buffer_rsrc_t rin, __amdgpu_buffer_rsrc_t rom,
                                       bool act, float (&r)[8], uint32_t &j4) {
    const uint32_t j = R.pre + (uint32_t)mbcnt64(R.m);
    const uint32_t a = pbyte(j);
    j4 = act ? a : kOutOfRange;
    const uint32_t o1 = lane_sel(R.left, pbyte(j - 1u) + 256u, a + 512u);
    const uint32_t o2 = lane_sel(R.right, pbyte(j + 1u) + 512u, a + 256u);
    const uint32_t o3 = lane_sel(R.nb[0], pbyte(R.pnb[0] + (uint32_t)mbcnt64(R.nb[0])) + 768u, a + 1024u);
    const uint32_t o4 = lane_sel(R.nb[1], pbyte(R.pnb[1] + (uint32_t)mbcnt64(R.nb[1])) + 1024u, a + 768u);
    const uint32_t o5 = lane_sel(R.nb[2], pbyte(R.pnb[2] + (uint32_t)mbcnt64(R.nb[2])) + 1280u, a + 1536u);
    const uint32_t o6 = lane_sel(R.nb[3], pbyte(R.pnb[3] + (uint32_t)mbcnt64(R.nb[3])) + 1536u, a + 1280u);
    r[0] = ld(rin, j4, 0);
    r[1] = ld(rin, act ? o1 : kOutOfRange, 0);
    r[2] = ld(rin, act ? o2 : kOutOfRange, 0);
    r[3] = ld(rin, act ? o3 : kOutOfRange, 0);
    r[4] = ld(rin, act ? o4 : kOutOfRange, 0);
    r[5] = ld(rin, act ? o5 : kOutOfRange, 0);
    r[6] = ld(rin, act ? o6 : kOutOfRange, 0);
    r[7] = KNUDSEN ? ld(rom, act ? 4u * j : kOutOfRange, 0) : 0.f;
}

// The same pulls as byte offsets (the relaxation rate's last), computed apart
// from the loads; past every buffer for lanes with nothing to do.
__device__ __forceinline__ void pull_offsets(const SegRec &R, bool act, uint32_t (&o)[8], uint32_t &j4) {
    const uint32_t j = R.pre + (uint32_t)mbcnt64(R.m);
    const uint32_t a = pbyte(j);
    j4 = act ? a : kOutOfRange;
    o[0] = j4;
    o[1] = act ? lane_sel(R.left, pbyte(j - 1u) + 256u, a + 512u) : kOutOfRange;
    o[2] = act ? lane_sel(R.right, pbyte(j + 1u) + 512u, a + 256u) : kOutOfRange;
    o[3] = act ? lane_sel(R.nb[0], pbyte(R.pnb[0] + (uint32_t)mbcnt64(R.nb[0])) + 768u, a + 1024u) : kOutOfRange;
    o[4] = act ? lane_sel(R.nb[1], pbyte(R.pnb[1] + (uint32_t)mbcnt64(R.nb[1])) + 1024u, a + 768u) : kOutOfRange;
    o[5] = act ? lane_sel(R.nb[2], pbyte(R.pnb[2] + (uint32_t)mbcnt64(R.nb[2])) + 1280u, a + 1536u) : kOutOfRange;
    o[6] = act ? lane_sel(R.nb[3], pbyte(R.pnb[3] + (uint32_t)mbcnt64(R.nb[3])) + 1536u, a + 1280u) : kOutOfRange;
    o[7] = act ? 4u * j : kOutOfRange;
}

// The eight loads of pull_offsets, issued without waiting.
template <bool KNUDSEN>
__device__ __forceinline__ void pull_loads(__amdgpu_buffer_rsrc_t rin, __amdgpu_buffer_rsrc_t rom,
                                           const uint32_t (&o)[8], float (&r)[8]) {
#pragma unroll
    for (int i = 0; i < 7; ++i) r[i] = ld(rin, o[i], 0);
    r[7] = KNUDSEN ? ld(rom, o[7], 0) : 0.f;
}

// Collision of one voxel in FP64 from its seven pulled stored values: x faces
// (anti-bounce-back Dirichlet at the inlet; Dirichlet or zero-gradient outlet),
// re-referencing of the +-x pulls to this voxel's shift, the sink -k n C, and the
// seven post-collision values rounded once to FP32.  left/right: the x -+ 1
// neighbour is fluid; n: catalyst face-neighbour count of a reacting voxel.
template <bool REACT>
__device__ __forceinline__ void collide7(const InstDev &I, int x, bool left, bool right, double om, int n,
                                         const float (&r)[8], float (&o)[7]) {
    const double p0 = r[0], p3 = r[3], p4 = r[4], p5 = r[5], p6 = r[6];
    double p1 = left ? (double)r[1] + I.pull_dx : (double)r[1];
    double p2 = right ? (double)r[2] - I.pull_dx : (double)r[2];
    if (x == 0) p1 = I.abb_in - (double)r[1];
    if (!REACT && x == I.nx - 1) p2 = I.abb_out - (double)r[2];

    const double Cs = ((p0 + p1) + (p2 + p3)) + ((p4 + p5) + p6);  // C - c_sh(x), exact
    double s0 = 0.0, s1 = 0.0;
    if (REACT) {
        const double kn = I.k * (double)n;
        const double sink = -kn * (Cs + (I.sh0 - I.slope * (double)x));
        s0 = I.w0 * sink;
        s1 = I.w1 * sink;
    }
    const double e0 = I.w0 * Cs, e1 = I.w1 * Cs;
    o[0] = (float)(fma(om, e0 - p0, p0) + s0);
    o[1] = (float)(fma(om, e1 - p1, p1) + s1);
    o[2] = (float)(fma(om, e1 - p2, p2) + s1);
    o[3] = (float)(fma(om, e1 - p3, p3) + s1);
    o[4] = (float)(fma(om, e1 - p4, p4) + s1);
    o[5] = (float)(fma(om, e1 - p5, p5) + s1);
    o[6] = (float)(fma(om, e1 - p6, p6) + s1);
}

// Relaxation rate of a lane: stored per voxel (Knudsen) or from the phase.
template <bool KNUDSEN>
__device__ __forceinline__ double lane_omega(const SegRec &R, const InstDev &I, float stored) {
    if (KNUDSEN) return (double)stored;
    return (double)__uint_as_float(lane_sel(R.ion, __float_as_uint(I.om_ion), __float_as_uint(I.om_pore)));
}

// Collide phase of one segment: FP64 collision with the sink, seven FP32 stores.
template <bool KNUDSEN, bool REACT>
__device__ __forceinline__ void collide_store(const SegRec &R, const InstDev &I, __amdgpu_buffer_rsrc_t rout,
                                              int lane, const float (&r)[8], uint32_t j4) {
    float o[7];
    collide7<REACT>(I, lane_x(R, lane), bit(R.left, lane), bit(R.right, lane), lane_omega<KNUDSEN>(R, I, r[7]),
                    REACT ? react_n(R, lane) : 0, r, o);
#pragma unroll
    for (int i = 0; i < 7; ++i) st(o[i], rout, j4, 256u * i);
}

// Fused pull stream + collide.  Each wave takes SPW consecutive list entries (row
// segments holding fluid) and issues all their loads before any arithmetic, so a
// wave keeps SPW x 8 loads in flight.
template <int WAVES, int SPW, bool KNUDSEN, bool REACT, bool SINGLE>
__global__ __launch_bounds__(WAVES * 64) void k_step(Lattice L, StepLaunch S, const float *__restrict__ fin,
                                                    float *__restrict__ fout) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int b = S.reverse ? logical_block_reversed(blockIdx.x, S.nblk, S.xcd) : logical_block(blockIdx.x, S.nblk, S.xcd);
    const uint32_t S4 = 4u * L.stride;
    const __amdgpu_buffer_rsrc_t rin = rsrc(fin, 7u * S4), rout = rsrc(fout, 7u * S4);
    const __amdgpu_buffer_rsrc_t rom = rsrc(L.omega, KNUDSEN ? S4 : 0u);
    const int base = (b * WAVES + wave) * SPW;
    const SegRec *R[SPW];
    const InstDev *Ip[SPW];
    bool act[SPW];
    float r[SPW][8];
    uint32_t j4[SPW];
#pragma unroll
    for (int k = 0; k < SPW; ++k) {
        const bool valid = base + k < S.nent;  // wave-uniform
        const int idx = valid ? base + k : 0;
        R[k] = &L.rec[S.list[idx]];
        Ip[k] = &L.inst[SINGLE ? 0 : S.list_inst[idx]];  // independent of the record
        act[k] = valid && bit(R[k]->m, lane);
        gather<KNUDSEN>(*R[k], rin, rom, act[k], r[k], j4[k]);
    }
#pragma unroll
    for (int k = 0; k < SPW; ++k) {
        if (act[k]) collide_store<KNUDSEN, REACT>(*R[k], *Ip[k], rout, lane, r[k], j4[k]);
    }
}

// ------------------------------------------------------------------ two steps per pass

// Per-lane bits of one voxel kept between issuing its loads and its collisions.
enum : uint32_t { F_ACT = 1u, F_LEFT = 2u, F_RIGHT = 4u, F_NB = 8u /* 4 bits */, F_ION = 128u, F_N = 8u /* shift */ };

__device__ __forceinline__ uint32_t lane_flags(const SegRec &R, int lane) {
    return (uint32_t)bit(R.m, lane) | (uint32_t)bit(R.left, lane) << 1 | (uint32_t)bit(R.right, lane) << 2 |
           (uint32_t)bit(R.nb[0], lane) << 3 | (uint32_t)bit(R.nb[1], lane) << 4 | (uint32_t)bit(R.nb[2], lane) << 5 |
           (uint32_t)bit(R.nb[3], lane) << 6 | (uint32_t)bit(R.ion, lane) << 7 | (uint32_t)react_n(R, lane) << F_N;
}

__device__ __forceinline__ double flag_omega(uint32_t fl, const InstDev &I, float stored, bool knudsen) {
    return knudsen ? (double)stored : (double)((fl & F_ION) ? I.om_ion : I.om_pore);
}

// Workgroup barrier ordering LDS only: this wave's LDS accesses are complete,
// its global loads and stores may still be in flight.
__device__ __forceinline__ void sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One step of the voxel just outside a segment's x range, one voxel per lane with
// its own record R: lane 63 of segment sn when side is 0 (the voxel before the
// range), lane 0 of segment sn when side is 1 (the voxel after it).  Returns the
// post-collision value that streams back into the range (+x, or -x), or 0 when the
// voxel is not simulated.
template <bool KNUDSEN, bool REACT>
__device__ __forceinline__ float edge_value(const SegRec *__restrict__ R, int side, int sn, const InstDev &I,
                                            __amdgpu_buffer_rsrc_t rin, __amdgpu_buffer_rsrc_t rom) {
    const int ln = side ? 0 : 63;
    const uint64_t below = side ? 0ull : ~0ull >> 1;  // lanes under ln
    const uint64_t m = R->m, left = R->left, right = R->right, ion = R->ion;
    const uint64_t nb0 = R->nb[0], nb1 = R->nb[1], nb2 = R->nb[2], nb3 = R->nb[3];
    const uint64_t n0 = R->n0, n1 = R->n1, n2 = R->n2;
    const uint32_t pre = R->pre, q0 = R->pnb[0], q1 = R->pnb[1], q2 = R->pnb[2], q3 = R->pnb[3];
    if (!bit(m, ln)) return 0.f;
    const uint32_t j = pre + (uint32_t)__popcll(m & below);
    const uint32_t a = pbyte(j);
    const uint64_t nb[4] = {nb0, nb1, nb2, nb3};
    const uint32_t pq[4] = {q0, q1, q2, q3};
    uint32_t o[7];
    o[0] = a;
    o[1] = bit(left, ln) ? pbyte(j - 1u) + 256u : a + 512u;
    o[2] = bit(right, ln) ? pbyte(j + 1u) + 512u : a + 256u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t own = a + 256u * (uint32_t)(k ^ 1) + 768u;  // bounce-back: the opposite population
        o[3 + k] = bit(nb[k], ln) ? pbyte(pq[k] + (uint32_t)__popcll(nb[k] & below)) + 768u + 256u * (uint32_t)k : own;
    }
    float r[8];
#pragma unroll
    for (int i = 0; i < 7; ++i) r[i] = ld(rin, o[i], 0);
    r[7] = KNUDSEN ? ld(rom, 4u * j, 0) : 0.f;
    const double om = KNUDSEN ? (double)r[7] : (double)(bit(ion, ln) ? I.om_ion : I.om_pore);
    const int n = REACT ? bit(n0, ln) + 2 * bit(n1, ln) + 4 * bit(n2, ln) : 0;
    float out[7];
    collide7<REACT>(I, sn * 64 + ln, bit(left, ln), bit(right, ln), om, n, r, out);
    return side ? out[2] : out[1];
}

// Loads of one row's first step in flight: the pulled values, the lane's flags and
// its own byte offset.
struct Pending {
    float g[8];
    uint32_t fl, j4;
};

constexpr int kStep2MaxPlanes = 64;  // planes per chunk (the x-edge table lives in LDS)

// Two steps per launch for one instance (see Step2Launch).  Block b (after the
// XCD renumbering) owns segment column s = b % nsx, rows y0 .. y0 + nr - 1 and
// planes z_lo .. z_hi - 1.
//   * First, every thread steps voxels just outside the x range (x0 - 1 and x0 + 64
//     of each tile row, planes z_lo - 1 .. z_hi) into an LDS table.
//   * Then iteration p (p = z_lo - 1 .. z_hi; planes wrap periodically) completes
//     the first step of plane p into LDS from loads issued two iterations earlier,
//     issues the loads of plane p + 2, and performs the second step of plane p - 1
//     from LDS into fout.
// Waves 0 .. BY - 1 own one tile row each; wave BY steps the row before the tile,
// wave BY + 1 the row after it.  Every value entering the second step is the FP32
// value the single-step kernel would have stored, so one launch of this kernel and
// two of that one give bit-identical lattices.
// At most 72 VGPRs (7 waves per SIMD): three 6-row or four 4-row workgroups per CU.
template <int BY, bool KNUDSEN, bool REACT>
__global__ __launch_bounds__((BY + 2) * 64) __attribute__((amdgpu_waves_per_eu(7))) void k_step2(
    Lattice L, Step2Launch S, const float *__restrict__ fin, float *__restrict__ fout) {
    __shared__ float full[2][BY][8][64];  // first step of a plane: 7 populations (+ 1/tau) per tile row
    __shared__ float zm[BY][64];          // +z population of the plane below the one in its second step
    __shared__ float yh[2][2][64];        // +y population of row y0 - 1, -y population of row y0 + nr
    __shared__ float xe[kStep2MaxPlanes + 2][BY][2];  // +x from x0 - 1, -x from x0 + 64, per plane and tile row
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const InstDev &I = L.inst[0];
    const int nsx = I.nsx, ny = I.ny, nz = I.nz;
    const int lb = logical_block(blockIdx.x, S.nblk, S.xcd);
    const int s = lb % nsx, t = lb / nsx;
    const int y0 = (t % S.nty) * BY, nr = min(BY, ny - y0);
    const int z_lo = (t / S.nty) * S.zc, z_hi = min(z_lo + S.zc, nz);
    const bool whole_y = nr == ny;  // the tile's own rows are its y neighbours
    const uint32_t S4 = 4u * L.stride;
    const __amdgpu_buffer_rsrc_t rin = rsrc(fin, 7u * S4), rout = rsrc(fout, 7u * S4);
    const __amdgpu_buffer_rsrc_t rom = rsrc(L.omega, KNUDSEN ? S4 : 0u);
    const int64_t plane_stride = (int64_t)ny * nsx;

    // ---- x-edge voxels of every plane of the chunk (task = (plane, tile row, side))
    const int ntask = (z_hi - z_lo + 2) * nr * 2;
    for (int task = (int)threadIdx.x; task < ntask; task += (BY + 2) * 64) {
        const int side = task & 1, tr = (task >> 1) % nr, pi = (task >> 1) / nr;
        const int sn = side ? s + 1 : s - 1;
        float v = 0.f;
        if (sn >= 0 && sn < nsx) {
            const int p = z_lo - 1 + pi;
            const int zp = p < 0 ? p + nz : (p >= nz ? p - nz : p);
            v = edge_value<KNUDSEN, REACT>(L.rec + zp * plane_stride + (int64_t)(y0 + tr) * nsx + sn, side, sn, I, rin,
                                           rom);
        }
        xe[pi][tr][side] = v;
    }

    // This wave's row: 0 tile row, 1 the row before the tile, 2 the row after it, -1 none.
    int kind = -1, row = 0;
    if (wave < nr) {
        kind = 0;
        row = y0 + wave;
    } else if (!whole_y && wave == BY) {
        kind = 1;
        row = y0 == 0 ? ny - 1 : y0 - 1;
    } else if (!whole_y && wave == BY + 1) {
        kind = 2;
        row = y0 + nr == ny ? 0 : y0 + nr;
    }
    const SegRec *Rrow = L.rec + (int64_t)row * nsx + s;
    // Every wave issues the same eight loads and seven stores in every iteration
    // (offsets past the buffers where there is nothing to do), so the compiler's
    // wait counts stay exact across the loop and the next planes' loads stay in
    // flight while a plane is consumed.
    auto issue = [&](int p, Pending &P) {
        uint32_t o[8];
        if (kind >= 0 && p <= z_hi) {
            const int zp = p < 0 ? p + nz : (p >= nz ? p - nz : p);
            const SegRec &R = Rrow[zp * plane_stride];
            P.fl = lane_flags(R, lane);
            pull_offsets(R, (P.fl & F_ACT) != 0, o, P.j4);
        } else {
            P.fl = 0;
            P.j4 = kOutOfRange;
#pragma unroll
            for (int i = 0; i < 8; ++i) o[i] = kOutOfRange;
        }
        pull_loads<KNUDSEN>(rin, rom, o, P.g);
    };
    uint32_t flq = 0, j4q = kOutOfRange;  // the plane in its second step
    // iteration p: first step of plane p from P, loads of plane p + 2 into P, second
    // step of plane p - 1
    auto iterate = [&](int p, Pending &P) {
        const int ps = p & 1;
        if (kind >= 0 && (P.fl & F_ACT)) {
            float o[7];
            collide7<REACT>(I, s * 64 + lane, (P.fl & F_LEFT) != 0, (P.fl & F_RIGHT) != 0,
                            flag_omega(P.fl, I, P.g[7], KNUDSEN), REACT ? (int)(P.fl >> F_N) : 0, P.g, o);
            if (kind == 0) {
#pragma unroll
                for (int i = 0; i < 7; ++i) full[ps][wave][i][lane] = o[i];
                if (KNUDSEN) full[ps][wave][7][lane] = P.g[7];
            } else {
                yh[ps][kind - 1][lane] = kind == 1 ? o[3] : o[4];
            }
        }
        const uint32_t flp = P.fl, j4p = P.j4;
        issue(p + 2, P);
        sync_lds();
        const int q = p - 1, qs = q & 1;
        const bool second = kind == 0 && q >= z_lo && (flq & F_ACT);
        float o[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (second) {
            const float(&F)[BY][8][64] = full[qs];
            const int qi = q - (z_lo - 1);
            float r[8];
            r[0] = F[wave][0][lane];
            r[1] = (flq & F_LEFT) ? (lane > 0 ? F[wave][1][lane - 1] : xe[qi][wave][0]) : F[wave][2][lane];
            r[2] = (flq & F_RIGHT) ? (lane < 63 ? F[wave][2][lane + 1] : xe[qi][wave][1]) : F[wave][1][lane];
            r[3] = (flq & (F_NB << 0))
                       ? (wave > 0 ? F[wave - 1][3][lane] : (whole_y ? F[nr - 1][3][lane] : yh[qs][0][lane]))
                       : F[wave][4][lane];
            r[4] = (flq & (F_NB << 1))
                       ? (wave + 1 < nr ? F[wave + 1][4][lane] : (whole_y ? F[0][4][lane] : yh[qs][1][lane]))
                       : F[wave][3][lane];
            r[5] = (flq & (F_NB << 2)) ? zm[wave][lane] : F[wave][6][lane];
            r[6] = (flq & (F_NB << 3)) ? full[ps][wave][6][lane] : F[wave][5][lane];
            r[7] = KNUDSEN ? F[wave][7][lane] : 0.f;
            collide7<REACT>(I, s * 64 + lane, (flq & F_LEFT) != 0, (flq & F_RIGHT) != 0,
                            flag_omega(flq, I, r[7], KNUDSEN), REACT ? (int)(flq >> F_N) : 0, r, o);
        }
        const uint32_t jst = second ? j4q : kOutOfRange;
#pragma unroll
        for (int i = 0; i < 7; ++i) st(o[i], rout, jst, 256u * i);
        if (kind == 0 && q >= z_lo - 1 && (flq & F_ACT)) zm[wave][lane] = full[qs][wave][5][lane];
        flq = flp;
        j4q = j4p;
        sync_lds();
    };

    // the prologue issues the loop's sequence of memory operations: the loads, then
    // seven (dropped) stores, per plane
    auto no_stores = [&]() {
#pragma unroll
        for (int i = 0; i < 7; ++i) st(0.f, rout, kOutOfRange, 256u * i);
    };
    Pending A, B;
    issue(z_lo - 1, A);
    no_stores();
    issue(z_lo, B);  // z_lo < z_hi
    no_stores();
    sync_lds();  // the x-edge table is complete
    int p = z_lo - 1;
    for (; p + 1 <= z_hi; p += 2) {  // both halves unconditional: exact wait counts at the back-edge
        iterate(p, A);
        iterate(p + 1, B);
    }
    if (p <= z_hi) iterate(p, A);
}

// ------------------------------------------------------------------ FP64 reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

constexpr int kMeasWaves = 4;

// Fluxes of the next streaming, sink and mass of the stored post-collision state
// (the same quantities the steady-state outputs use), per instance, in FP64.
template <bool REACT>
__global__ __launch_bounds__(kMeasWaves * 64) void k_measure(Lattice L, MeasureLaunch M, const float *__restrict__ f) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int4 t = M.blk[blockIdx.x];
    const InstDev &I = L.inst[t.x];
    double acc[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) acc[i] = 0.0;
    for (int64_t sl = (int64_t)t.y * kMeasWaves + wave; sl < I.nseg; sl += (int64_t)t.z * kMeasWaves) {
        const SegRec &R = L.rec[I.seg_base + sl];
        const uint64_t m = R.m;
        if (m == 0ull) continue;
        if (!bit(m, lane)) continue;
        const int64_t j = (int64_t)R.pre + mbcnt64(m);
        const int x = lane_x(R, lane);
        double cs = 0.0;
#pragma unroll
        for (int i = 0; i < 7; ++i) cs += (double)f[pidx(i, j)];
        const double kn = REACT ? I.k * react_n(R, lane) : 0.0;
        const double C = (cs + (I.sh0 - I.slope * (double)x)) / (1.0 - kn);
        acc[Q_MASS] += C;
        acc[Q_RATE] += kn * C;
        if (x == 0) acc[Q_JIN] += I.abb_in - 2.0 * (double)f[pidx(2, j)];
        if (!REACT && x == I.nx - 1) acc[Q_JOUT] += 2.0 * (double)f[pidx(1, j)] - I.abb_out;
        // link flux f*_{+x}(x) - f*_{-x}(x+1); the shifts differ by w1 * slope
        if (bit(R.right, lane)) acc[Q_JINT] += (double)f[pidx(1, j)] - (double)f[pidx(2, j + 1)] + I.pull_dx;
        const double dc = fabs(C - (double)M.csnap[j]);
        acc[Q_DCMAX] = fmax(acc[Q_DCMAX], dc);
        acc[Q_CMAX] = fmax(acc[Q_CMAX], fabs(C));
        if (!isfinite(C)) acc[Q_BAD] += 1.0;
        if (M.update_snap) M.csnap[j] = (float)C;
    }
    __shared__ double red[kMeasWaves][NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const double v = (i == Q_DCMAX || i == Q_CMAX) ? wave_max(acc[i]) : wave_sum(acc[i]);
        if (lane == 0) red[wave][i] = v;
    }
    __syncthreads();
    if (threadIdx.x < NQ) {
        const int i = threadIdx.x;
        double v = red[0][i];
        for (int w = 1; w < kMeasWaves; ++w) v = (i == Q_DCMAX || i == Q_CMAX) ? fmax(v, red[w][i]) : v + red[w][i];
        M.partial[(int64_t)t.w * NQ + i] = v;
    }
}

// Per-instance totals of the reduction partials: 64 threads stride over the
// instance's partial slots, then a fixed-order wave reduction (deterministic).
__global__ __launch_bounds__(64) void k_finish(const double *__restrict__ partial, const int2 *__restrict__ ranges,
                                               double *results) {
    const int inst = blockIdx.x;
    const int lane = threadIdx.x;
    const int2 r = ranges[inst];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const bool mx = (i == Q_DCMAX || i == Q_CMAX);
        double v = 0.0;
        for (int b = lane; b < r.y; b += 64) {
            const double p = partial[(int64_t)(r.x + b) * NQ + i];
            v = mx ? fmax(v, p) : v + p;
        }
        v = mx ? wave_max(v) : wave_sum(v);
        if (lane == 0) results[(int64_t)inst * NQ + i] = v;
    }
}

// ------------------------------------------------------------------ conversions

// Calls fn(instance, I, dense voxel index v, compact index j or -1, catalyst count
// of reacting lanes) for every lane of the segment that lies inside the grid.
template <typename Fn>
__device__ __forceinline__ void for_lanes(const Lattice &L, const int2 *blk, Fn fn) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int2 t = blk[blockIdx.x];
    const InstDev &I = L.inst[t.x];
    const int64_t sl = (int64_t)t.y + wave;
    if (sl >= I.nseg) return;
    const SegRec &R = L.rec[I.seg_base + sl];
    if (lane >= (int)R.len) return;
    const int64_t v = (int64_t)R.v0 + lane;
    const bool fluid = bit(R.m, lane);
    const int64_t j = fluid ? (int64_t)R.pre + mbcnt64(R.m) : -1;
    fn(t.x, I, v, j, (double)react_n(R, lane));
}

__global__ __launch_bounds__(256) void k_init_eq(Lattice L, const int2 *blk, int react, const float *c_dense,
                                                const int64_t *dbase, float *f, float *csnap) {
    for_lanes(L, blk, [&](int inst, const InstDev &I, int64_t v, int64_t j, double n) {
        if (j < 0) return;
        const double C = c_dense ? (double)c_dense[dbase[inst] + v] : 0.0;
        const double kn = react ? I.k * n : 0.0;
        const int x = (int)(v % I.nx);
        const double post = C * (1.0 - kn) - (I.sh0 - I.slope * x);  // equilibrium after the sink, shifted
        f[pidx(0, j)] = (float)(I.w0 * post);
        for (int i = 1; i < 7; ++i) f[pidx(i, j)] = (float)(I.w1 * post);
        csnap[j] = (float)C;
    });
}

__global__ __launch_bounds__(256) void k_set_pop(Lattice L, const int2 *blk, const float *fd, const int64_t *dbase,
                                                int64_t dstride, float *f) {
    for_lanes(L, blk, [&](int inst, const InstDev &I, int64_t v, int64_t j, double) {
        if (j < 0) return;
        const int64_t d = dbase[inst] + v;
        const double sh = I.sh0 - I.slope * (double)(v % I.nx);
        f[pidx(0, j)] = (float)((double)fd[d] - I.w0 * sh);
        for (int i = 1; i < 7; ++i) f[pidx(i, j)] = (float)((double)fd[i * dstride + d] - I.w1 * sh);
    });
}

__global__ __launch_bounds__(256) void k_get_pop(Lattice L, const int2 *blk, const float *f, const int64_t *dbase,
                                                int64_t dstride, float *fd) {
    for_lanes(L, blk, [&](int inst, const InstDev &I, int64_t v, int64_t j, double) {
        const int64_t d = dbase[inst] + v;
        const double sh = I.sh0 - I.slope * (double)(v % I.nx);
        for (int i = 0; i < 7; ++i) {
            const double w = i == 0 ? I.w0 : I.w1;
            fd[i * dstride + d] = j < 0 ? 0.f : (float)((double)f[pidx(i, j)] + w * sh);
        }
    });
}

__global__ __launch_bounds__(256) void k_conc(Lattice L, const int2 *blk, int react, const float *f,
                                             const int64_t *dbase, float *c) {
    for_lanes(L, blk, [&](int inst, const InstDev &I, int64_t v, int64_t j, double n) {
        float out = 0.f;
        if (j >= 0) {
            double cs = 0.0;
            for (int i = 0; i < 7; ++i) cs += (double)f[pidx(i, j)];
            const double kn = react ? I.k * n : 0.0;
            out = (float)((cs + (I.sh0 - I.slope * (double)(v % I.nx))) / (1.0 - kn));
        }
        c[dbase[inst] + v] = out;
    });
}

template <int W, int SPW, bool SINGLE>
hipError_t launch_step_t(const Lattice &L, const StepLaunch &S, bool kn, bool re, const float *fin, float *fout,
                         hipStream_t st) {
    const dim3 grid(S.nblk), block(W * 64);
    (void)hipGetLastError();  // drop a stale error (e.g. hipErrorNotReady from an event query)
    if (kn && re) {
        hipLaunchKernelGGL((k_step<W, SPW, true, true, SINGLE>), grid, block, 0, st, L, S, fin, fout);
    } else if (kn) {
        hipLaunchKernelGGL((k_step<W, SPW, true, false, SINGLE>), grid, block, 0, st, L, S, fin, fout);
    } else if (re) {
        hipLaunchKernelGGL((k_step<W, SPW, false, true, SINGLE>), grid, block, 0, st, L, S, fin, fout);
    } else {
        hipLaunchKernelGGL((k_step<W, SPW, false, false, SINGLE>), grid, block, 0, st, L, S, fin, fout);
    }
    return hipGetLastError();
}

template <int W, int SPW>
hipError_t launch_step_s(const Lattice &L, const StepLaunch &S, bool kn, bool re, const float *fin, float *fout,
                         hipStream_t st) {
    return S.single ? launch_step_t<W, SPW, true>(L, S, kn, re, fin, fout, st)
                    : launch_step_t<W, SPW, false>(L, S, kn, re, fin, fout, st);
}

template <int W>
hipError_t launch_step_w(const Lattice &L, const StepLaunch &S, bool kn, bool re, const float *fin, float *fout,
                         hipStream_t st) {
    switch (S.spw) {
        case 1: return launch_step_s<W, 1>(L, S, kn, re, fin, fout, st);
        case 2: return launch_step_s<W, 2>(L, S, kn, re, fin, fout, st);
        case 4: return launch_step_s<W, 4>(L, S, kn, re, fin, fout, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_step(const Lattice &L, const StepLaunch &S, bool knudsen, bool react, const float *fin,
                       float *fout, hipStream_t st) {
    if (S.nblk <= 0) return hipSuccess;
    switch (S.waves) {
        case 1: return launch_step_w<1>(L, S, knudsen, react, fin, fout, st);
        case 2: return launch_step_w<2>(L, S, knudsen, react, fin, fout, st);
        case 4: return launch_step_w<4>(L, S, knudsen, react, fin, fout, st);
        case 8: return launch_step_w<8>(L, S, knudsen, react, fin, fout, st);
        default: return hipErrorInvalidValue;
    }
}

namespace {
template <int BY>
hipError_t launch_step2_t(const Lattice &L, const Step2Launch &S, bool kn, bool re, const float *fin, float *fout,
                          hipStream_t st) {
    const dim3 grid(S.nblk), block((BY + 2) * 64);
    (void)hipGetLastError();
    if (kn && re) {
        hipLaunchKernelGGL((k_step2<BY, true, true>), grid, block, 0, st, L, S, fin, fout);
    } else if (kn) {
        hipLaunchKernelGGL((k_step2<BY, true, false>), grid, block, 0, st, L, S, fin, fout);
    } else if (re) {
        hipLaunchKernelGGL((k_step2<BY, false, true>), grid, block, 0, st, L, S, fin, fout);
    } else {
        hipLaunchKernelGGL((k_step2<BY, false, false>), grid, block, 0, st, L, S, fin, fout);
    }
    return hipGetLastError();
}
}  // namespace

hipError_t launch_step2(const Lattice &L, const Step2Launch &S, bool knudsen, bool react, const float *fin,
                        float *fout, hipStream_t st) {
    if (S.zc < 1 || S.zc > kStep2MaxPlanes) return hipErrorInvalidValue;  // the x-edge table's planes
    if (S.nblk <= 0) return hipSuccess;
    switch (S.by) {
        case 4: return launch_step2_t<4>(L, S, knudsen, react, fin, fout, st);
        case 6: return launch_step2_t<6>(L, S, knudsen, react, fin, fout, st);
        case 8: return launch_step2_t<8>(L, S, knudsen, react, fin, fout, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_measure(const Lattice &L, const MeasureLaunch &M, bool react, const float *f, hipStream_t st) {
    if (M.nblk <= 0) return hipSuccess;
    (void)hipGetLastError();
    if (react) {
        hipLaunchKernelGGL(k_measure<true>, dim3(M.nblk), dim3(kMeasWaves * 64), 0, st, L, M, f);
    } else {
        hipLaunchKernelGGL(k_measure<false>, dim3(M.nblk), dim3(kMeasWaves * 64), 0, st, L, M, f);
    }
    return hipGetLastError();
}

hipError_t launch_finish(const double *partial, const int2 *ranges, int32_t ninst, double *results, hipStream_t st) {
    if (ninst <= 0) return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_finish, dim3(ninst), dim3(64), 0, st, partial, ranges, results);
    return hipGetLastError();
}

hipError_t launch_init_eq(const Lattice &L, int32_t nblk, const int2 *blk, bool react, const float *c_dense,
                          const int64_t *dense_base, float *f, float *csnap, hipStream_t st) {
    if (nblk <= 0) return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_init_eq, dim3(nblk), dim3(256), 0, st, L, blk, react ? 1 : 0, c_dense, dense_base, f, csnap);
    return hipGetLastError();
}

hipError_t launch_set_pop(const Lattice &L, int32_t nblk, const int2 *blk, const float *f_dense,
                          const int64_t *dense_base, int64_t dense_stride, float *f, hipStream_t st) {
    if (nblk <= 0) return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_set_pop, dim3(nblk), dim3(256), 0, st, L, blk, f_dense, dense_base, dense_stride, f);
    return hipGetLastError();
}

hipError_t launch_get_pop(const Lattice &L, int32_t nblk, const int2 *blk, const float *f,
                          const int64_t *dense_base, int64_t dense_stride, float *f_dense, hipStream_t st) {
    if (nblk <= 0) return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_get_pop, dim3(nblk), dim3(256), 0, st, L, blk, f, dense_base, dense_stride, f_dense);
    return hipGetLastError();
}

hipError_t launch_conc(const Lattice &L, int32_t nblk, const int2 *blk, bool react, const float *f,
                       const int64_t *dense_base, float *c_dense, hipStream_t st) {
    if (nblk <= 0) return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_conc, dim3(nblk), dim3(256), 0, st, L, blk, react ? 1 : 0, f, dense_base, c_dense);
    return hipGetLastError();
}

}  // namespace cl
