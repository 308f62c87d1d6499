// D3Q7 reactive-diffusion lattice Boltzmann kernels for CDNA4 (gfx950).
//
// Scheme: Chen et al., arXiv 1410.1914, Section 4, Eq. (21) with g_eq = w_i C
// (Eq. 23 read on D3Q7), C = sum_i g_i (Eq. 24), sink S = -k n C (Eqs. 17b, 18a);
// boundaries of Section 3.5 (Eqs. 19, 20a, 20b).
//
// Layout (one wave64 = one 64-voxel row segment = one 64-bit mask word):
//   * m_fluid[seg] bit l is set when voxel (64 s + l, y, z) is simulated.
//   * Fluid voxels are stored compactly in x-fastest order; the compact index of a
//     fluid lane is prefix[seg] + mbcnt(m_fluid[seg]) (count of fluid lanes below it).
//   * The compact index of the +-y / +-z neighbour is found the same way from the
//     neighbour row's mask word and prefix, so no per-voxel neighbour table exists.
//   * Populations are SoA: f[i * stride + j], i = rest, +x, -x, +y, -y, +z, -z, stored
//     post-collision as g_i = f_i - w_i c_sh(x), c_sh the linear empty-box profile
//     (a constant for the reactive problem).  The shift is exact; it keeps the stored
//     values small so FP32 storage resolves the fluxes.
//   * Arithmetic is FP64: the seven FP32 loads are summed exactly, and each stored
//     value carries a single rounding, so rounding does not bias the mass balance.
//
// Every stored value is read exactly once per step (by the voxel it streams into,
// or by its own voxel when bounced back), and every fluid voxel writes its seven
// populations once: 56 bytes per fluid update plus the relaxation rate in Knudsen
// problems.  Solid voxels cost nothing but their share of the mask words.
#include "kernels.h"

namespace cl {
namespace {

__device__ __forceinline__ int mbcnt64(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int bit(uint64_t m, int lane) { return (int)((m >> lane) & 1ull); }

// Workgroups are dealt to the 8 XCDs round robin; renumber them so that each XCD
// works on one contiguous eighth of the grid (neighbour rows then share its L2).
__device__ __forceinline__ int logical_block(int b, int nblk, int remap) {
    if (!remap || nblk < 8) return b;
    const int q = nblk >> 3, r = nblk & 7;
    const int x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

struct Seg {
    int64_t g;             // global segment
    int s, y, z;
    int64_t gym, gyp, gzm, gzp;
};

__device__ __forceinline__ Seg locate(const InstDev &I, int64_t sl) {
    Seg q;
    q.s = (int)(sl % I.nsx);
    const int64_t row = sl / I.nsx;
    q.y = (int)(row % I.ny);
    q.z = (int)(row / I.ny);
    q.g = I.seg_base + sl;
    const int64_t rs = I.nsx, ps = (int64_t)I.ny * I.nsx;
    q.gym = q.g + (q.y == 0 ? (int64_t)(I.ny - 1) * rs : -rs);
    q.gyp = q.g + (q.y == I.ny - 1 ? -(int64_t)(I.ny - 1) * rs : rs);
    q.gzm = q.g + (q.z == 0 ? (int64_t)(I.nz - 1) * ps : -ps);
    q.gzp = q.g + (q.z == I.nz - 1 ? -(int64_t)(I.nz - 1) * ps : ps);
    return q;
}

// segment of a table entry: global index and periodic neighbour rows, no division
__device__ __forceinline__ Seg locate_entry(const InstDev &I, SegEntry e) {
    Seg q;
    q.s = e.s;
    q.y = e.y;
    q.z = e.z;
    const int64_t rs = I.nsx, ps = (int64_t)I.ny * I.nsx;
    q.g = I.seg_base + (int64_t)q.z * ps + (int64_t)q.y * rs + q.s;
    q.gym = q.g + (q.y == 0 ? (int64_t)(I.ny - 1) * rs : -rs);
    q.gyp = q.g + (q.y == I.ny - 1 ? -(int64_t)(I.ny - 1) * rs : rs);
    q.gzm = q.g + (q.z == 0 ? (int64_t)(I.nz - 1) * ps : -ps);
    q.gzp = q.g + (q.z == I.nz - 1 ? -(int64_t)(I.nz - 1) * ps : ps);
    return q;
}

// catalyst face neighbours of the lane's voxel (Eq. 18a): x bounded, y/z periodic
__device__ __forceinline__ int catalyst_count(const Lattice &L, const Seg &q, int nsx, int lane) {
    const uint64_t c = L.m_cat[q.g];
    const uint64_t cp = q.s > 0 ? L.m_cat[q.g - 1] : 0ull;
    const uint64_t cn = q.s + 1 < nsx ? L.m_cat[q.g + 1] : 0ull;
    const uint64_t cl = (c << 1) | (cp >> 63);
    const uint64_t cr = (c >> 1) | (cn << 63);
    return bit(cl, lane) + bit(cr, lane) + bit(L.m_cat[q.gym], lane) + bit(L.m_cat[q.gyp], lane) +
           bit(L.m_cat[q.gzm], lane) + bit(L.m_cat[q.gzp], lane);
}

// One fused pull stream + collide for the fluid lanes of one row segment.
template <bool KNUDSEN, bool REACT>
__device__ __forceinline__ void step_segment(const Lattice &L, const InstDev &I, const Seg &q, int lane,
                                             const float *__restrict__ fin, float *__restrict__ fout) {
    const uint64_t m = L.m_fluid[q.g];
    if (m == 0ull) return;
    const uint64_t mp = q.s > 0 ? L.m_fluid[q.g - 1] : 0ull;
    const uint64_t mn = q.s + 1 < I.nsx ? L.m_fluid[q.g + 1] : 0ull;
    const uint64_t mym = L.m_fluid[q.gym], myp = L.m_fluid[q.gyp];
    const uint64_t mzm = L.m_fluid[q.gzm], mzp = L.m_fluid[q.gzp];
    const uint32_t pre = L.prefix[q.g];
    const uint32_t pym = L.prefix[q.gym], pyp = L.prefix[q.gyp];
    const uint32_t pzm = L.prefix[q.gzm], pzp = L.prefix[q.gzp];
    const uint64_t left = (m << 1) | (mp >> 63);   // bit l: voxel x-1 is fluid
    const uint64_t right = (m >> 1) | (mn << 63);  // bit l: voxel x+1 is fluid
    uint64_t mion = 0, mreact = 0;
    if (!KNUDSEN) mion = L.m_ion[q.g];
    if (REACT) mreact = L.m_react[q.g];
    int ncat = 0;
    if (REACT) ncat = catalyst_count(L, q, I.nsx, lane);

    if (!bit(m, lane)) return;
    const int64_t S = L.stride;
    const int64_t j = (int64_t)pre + mbcnt64(m);
    const int x = q.s * 64 + lane;

    // pull the seven populations (bounce-back reads the voxel's own opposite one)
    const bool fl = bit(left, lane), fr = bit(right, lane);
    const int64_t a1 = fl ? 1 * S + j - 1 : 2 * S + j;
    const int64_t a2 = fr ? 2 * S + j + 1 : 1 * S + j;
    const int64_t a3 = bit(mym, lane) ? 3 * S + (int64_t)pym + mbcnt64(mym) : 4 * S + j;
    const int64_t a4 = bit(myp, lane) ? 4 * S + (int64_t)pyp + mbcnt64(myp) : 3 * S + j;
    const int64_t a5 = bit(mzm, lane) ? 5 * S + (int64_t)pzm + mbcnt64(mzm) : 6 * S + j;
    const int64_t a6 = bit(mzp, lane) ? 6 * S + (int64_t)pzp + mbcnt64(mzp) : 5 * S + j;
    const float r0 = fin[j], r1 = fin[a1], r2 = fin[a2], r3 = fin[a3], r4 = fin[a4], r5 = fin[a5], r6 = fin[a6];
    const double p0 = r0, p3 = r3, p4 = r4, p5 = r5, p6 = r6;
    // +-x: re-reference to this voxel's shift; x faces: anti-bounce-back Dirichlet at
    // the inlet, Dirichlet (anti-bounce-back) or zero-gradient (bounce-back) outlet
    double p1 = fl ? (double)r1 + I.pull_dx : (double)r1;
    double p2 = fr ? (double)r2 - I.pull_dx : (double)r2;
    if (x == 0) p1 = I.abb_in - (double)r1;
    if (!REACT && x == I.nx - 1) p2 = I.abb_out - (double)r2;

    const double Cs = ((p0 + p1) + (p2 + p3)) + ((p4 + p5) + p6);  // C - c_sh(x), exact
    double om;
    if (KNUDSEN)
        om = (double)L.omega[j];
    else
        om = (double)(bit(mion, lane) ? I.om_ion : I.om_pore);
    double s0 = 0.0, s1 = 0.0;
    if (REACT) {
        const double kn = bit(mreact, lane) ? I.k * (double)ncat : 0.0;
        const double sink = -kn * (Cs + (I.sh0 - I.slope * (double)x));
        s0 = I.w0 * sink;
        s1 = I.w1 * sink;
    }
    const double e0 = I.w0 * Cs, e1 = I.w1 * Cs;
    fout[j] = (float)(fma(om, e0 - p0, p0) + s0);
    fout[1 * S + j] = (float)(fma(om, e1 - p1, p1) + s1);
    fout[2 * S + j] = (float)(fma(om, e1 - p2, p2) + s1);
    fout[3 * S + j] = (float)(fma(om, e1 - p3, p3) + s1);
    fout[4 * S + j] = (float)(fma(om, e1 - p4, p4) + s1);
    fout[5 * S + j] = (float)(fma(om, e1 - p5, p5) + s1);
    fout[6 * S + j] = (float)(fma(om, e1 - p6, p6) + s1);
}

template <int WAVES, int SPW, bool KNUDSEN, bool REACT>
__global__ __launch_bounds__(WAVES * 64) void k_step(Lattice L, const SegEntry *__restrict__ seg, int nent, int nblk,
                                                    int remap, const float *__restrict__ fin, float *__restrict__ fout) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int b = logical_block(blockIdx.x, nblk, remap);
#pragma unroll
    for (int k = 0; k < SPW; ++k) {
        const int idx = (b * WAVES + wave) * SPW + k;
        if (idx < nent) {
            const SegEntry e = seg[idx];
            const InstDev &I = L.inst[e.inst];
            step_segment<KNUDSEN, REACT>(L, I, locate_entry(I, e), lane, fin, fout);
        }
    }
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
    const int64_t S = L.stride;
    double acc[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) acc[i] = 0.0;
    for (int64_t sl = (int64_t)t.y * kMeasWaves + wave; sl < I.nseg; sl += (int64_t)t.z * kMeasWaves) {
        const Seg q = locate(I, sl);
        const uint64_t m = L.m_fluid[q.g];
        if (m == 0ull) continue;
        const uint64_t mn = q.s + 1 < I.nsx ? L.m_fluid[q.g + 1] : 0ull;
        const uint64_t right = (m >> 1) | (mn << 63);
        const uint32_t pre = L.prefix[q.g];
        int ncat = 0;
        uint64_t mreact = 0;
        if (REACT) {
            ncat = catalyst_count(L, q, I.nsx, lane);
            mreact = L.m_react[q.g];
        }
        if (!bit(m, lane)) continue;
        const int64_t j = (int64_t)pre + mbcnt64(m);
        const int x = q.s * 64 + lane;
        double cs = 0.0;
#pragma unroll
        for (int i = 0; i < 7; ++i) cs += (double)f[i * S + j];
        const double kn = (REACT && bit(mreact, lane)) ? I.k * ncat : 0.0;
        const double C = (cs + (I.sh0 - I.slope * (double)x)) / (1.0 - kn);
        acc[Q_MASS] += C;
        acc[Q_RATE] += kn * C;
        if (x == 0) acc[Q_JIN] += I.abb_in - 2.0 * (double)f[2 * S + j];
        if (!REACT && x == I.nx - 1) acc[Q_JOUT] += 2.0 * (double)f[1 * S + j] - I.abb_out;
        // link flux f*_{+x}(x) - f*_{-x}(x+1); the shifts differ by w1 * slope
        if (bit(right, lane)) acc[Q_JINT] += (double)f[1 * S + j] - (double)f[2 * S + j + 1] + I.pull_dx;
        const float Cf = (float)C;
        const double dc = fabs(C - (double)M.csnap[j]);
        acc[Q_DCMAX] = fmax(acc[Q_DCMAX], dc);
        acc[Q_CMAX] = fmax(acc[Q_CMAX], fabs(C));
        if (!isfinite(C)) acc[Q_BAD] += 1.0;
        if (M.update_snap) M.csnap[j] = Cf;
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

__global__ void k_finish(const double *__restrict__ partial, const int2 *__restrict__ ranges, double *results) {
    const int inst = blockIdx.x;
    const int i = threadIdx.x;
    if (i >= NQ) return;
    const int2 r = ranges[inst];
    double v = 0.0;
    for (int b = 0; b < r.y; ++b) {
        const double p = partial[(int64_t)(r.x + b) * NQ + i];
        v = (i == Q_DCMAX || i == Q_CMAX) ? fmax(v, p) : v + p;
    }
    results[(int64_t)inst * NQ + i] = v;
}

// ------------------------------------------------------------------ conversions

template <typename Fn>
__device__ __forceinline__ void for_lanes(const Lattice &L, const int2 *blk, Fn fn) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int2 t = blk[blockIdx.x];
    const InstDev &I = L.inst[t.x];
    const int64_t sl = (int64_t)t.y + wave;
    if (sl >= I.nseg) return;
    const Seg q = locate(I, sl);
    const uint64_t m = L.m_fluid[q.g];
    int ncat = 0;
    if (m) ncat = catalyst_count(L, q, I.nsx, lane);
    const uint64_t mreact = L.m_react[q.g];
    const int x = q.s * 64 + lane;
    if (x >= I.nx) return;
    const int64_t v = ((int64_t)q.z * I.ny + q.y) * I.nx + x;
    const bool fluid = bit(m, lane);
    const int64_t j = fluid ? (int64_t)L.prefix[q.g] + mbcnt64(m) : -1;
    fn(t.x, I, v, j, (double)ncat * bit(mreact, lane));
}

__global__ __launch_bounds__(256) void k_init_eq(Lattice L, const int2 *blk, int react, const float *c_dense,
                                                const int64_t *dbase, float *f, float *csnap) {
    for_lanes(L, blk, [&](int inst, const InstDev &I, int64_t v, int64_t j, double n) {
        if (j < 0) return;
        const double C = c_dense ? (double)c_dense[dbase[inst] + v] : 0.0;
        const double kn = react ? I.k * n : 0.0;
        const int x = (int)(v % I.nx);
        const double post = C * (1.0 - kn) - (I.sh0 - I.slope * x);  // equilibrium after the sink, shifted
        f[j] = (float)(I.w0 * post);
        for (int i = 1; i < 7; ++i) f[i * L.stride + j] = (float)(I.w1 * post);
        csnap[j] = (float)C;
    });
}

__global__ __launch_bounds__(256) void k_set_pop(Lattice L, const int2 *blk, const float *fd, const int64_t *dbase,
                                                int64_t dstride, float *f) {
    for_lanes(L, blk, [&](int inst, const InstDev &I, int64_t v, int64_t j, double) {
        if (j < 0) return;
        const int64_t d = dbase[inst] + v;
        const double sh = I.sh0 - I.slope * (double)(v % I.nx);
        f[j] = (float)((double)fd[d] - I.w0 * sh);
        for (int i = 1; i < 7; ++i) f[i * L.stride + j] = (float)((double)fd[i * dstride + d] - I.w1 * sh);
    });
}

__global__ __launch_bounds__(256) void k_get_pop(Lattice L, const int2 *blk, const float *f, const int64_t *dbase,
                                                int64_t dstride, float *fd) {
    for_lanes(L, blk, [&](int inst, const InstDev &I, int64_t v, int64_t j, double) {
        const int64_t d = dbase[inst] + v;
        const double sh = I.sh0 - I.slope * (double)(v % I.nx);
        for (int i = 0; i < 7; ++i) {
            const double w = i == 0 ? I.w0 : I.w1;
            fd[i * dstride + d] = j < 0 ? 0.f : (float)((double)f[i * L.stride + j] + w * sh);
        }
    });
}

__global__ __launch_bounds__(256) void k_conc(Lattice L, const int2 *blk, int react, const float *f,
                                             const int64_t *dbase, float *c) {
    for_lanes(L, blk, [&](int inst, const InstDev &I, int64_t v, int64_t j, double n) {
        float out = 0.f;
        if (j >= 0) {
            double cs = 0.0;
            for (int i = 0; i < 7; ++i) cs += (double)f[i * L.stride + j];
            const double kn = react ? I.k * n : 0.0;
            out = (float)((cs + (I.sh0 - I.slope * (double)(v % I.nx))) / (1.0 - kn));
        }
        c[dbase[inst] + v] = out;
    });
}

template <int W, int SPW>
hipError_t launch_step_t(const Lattice &L, const StepLaunch &S, bool kn, bool re, const float *fin, float *fout,
                         hipStream_t st) {
    const dim3 grid(S.nblk), block(W * 64);
    (void)hipGetLastError();  // drop a stale error (e.g. hipErrorNotReady from an event query)
    if (kn && re) {
        hipLaunchKernelGGL((k_step<W, SPW, true, true>), grid, block, 0, st, L, S.seg, S.nent, S.nblk, S.xcd, fin, fout);
    } else if (kn) {
        hipLaunchKernelGGL((k_step<W, SPW, true, false>), grid, block, 0, st, L, S.seg, S.nent, S.nblk, S.xcd, fin, fout);
    } else if (re) {
        hipLaunchKernelGGL((k_step<W, SPW, false, true>), grid, block, 0, st, L, S.seg, S.nent, S.nblk, S.xcd, fin, fout);
    } else {
        hipLaunchKernelGGL((k_step<W, SPW, false, false>), grid, block, 0, st, L, S.seg, S.nent, S.nblk, S.xcd, fin, fout);
    }
    return hipGetLastError();
}

template <int W>
hipError_t launch_step_w(const Lattice &L, const StepLaunch &S, bool kn, bool re, const float *fin, float *fout,
                         hipStream_t st) {
    switch (S.spw) {
        case 1: return launch_step_t<W, 1>(L, S, kn, re, fin, fout, st);
        case 2: return launch_step_t<W, 2>(L, S, kn, re, fin, fout, st);
        case 4: return launch_step_t<W, 4>(L, S, kn, re, fin, fout, st);
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
