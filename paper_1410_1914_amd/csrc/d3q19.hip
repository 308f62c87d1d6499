// D3Q19 variant of the solver: the lattice the paper itself uses (Chen et al.,
// arXiv 1410.1914, Section 4, Eqs. 21-24), beside the D3Q7 production path.
//
// Storage holds the simulated (fluid) voxels only, in x-fastest order: compact
// index j, populations in blocks of 64 compact voxels,
// f[(j >> 6) * 19 * 64 + i * 64 + (j & 63)], FP32, holding the post-collision
// value shifted by a_i * c_sh(x) (c_sh = sh0 - slope * x, the empty-box profile
// between Dirichlet faces, or half the inlet value when reacting), two lattices
// A/B.  A wave updates one segment, a window of up to 64 voxels consecutive in
// grid order cut as for the D3Q7 solver (each row into its own windows, or, for
// rows of 64 k + 1 voxels, windows running on across row ends within a plane, cut
// at rows 1 and ny - 1); its record (D19Rec) holds the fluid masks and compact
// prefixes of the nine windows it pulls from, the same lanes moved by (ry, rz)
// rows and planes for ry, rz in {-1, 0, 1}, so the compact index of any pull
// source is a prefix plus a count of mask bits, and no per-voxel neighbour table
// exists.
// Relaxation rates, sink coefficients and the concentration snapshot are compact
// too; a dense map from voxel to compact index serves the conversions.  The
// collision is evaluated in FP64 and rounded once to FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <vector>

#include "kernels.h"
#include "prep.h"

namespace {

constexpr int kQ = 19;
constexpr int kBlock = 256;
constexpr int kRed = 8;  // j_in, j_out, sum of interior face fluxes, rate, mass, max|dC|, max|C|, NaN count

// Eq. (22), in the order the public header documents: rest; +x, -x, +y, -y, +z,
// -z; the xy, xz and yz edges, each (+,+), (+,-), (-,+), (-,-).
constexpr int CX[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 0, 0, 0, 0};
constexpr int CY[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1};
constexpr int CZ[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
constexpr int OPP[kQ] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15};
// slot of a c_x = +1 direction among bits 19-23, of a c_x = -1 one among 24-28
constexpr int FACE_SLOT[kQ] = {-1, 0, 0, -1, -1, -1, -1, 1, 2, 1, 2, 3, 4, 3, 4, -1, -1, -1, -1};
constexpr uint32_t kActive = 1u << 31;

__host__ __device__ constexpr double weight(int i) { return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }

// Segment record of the compact layout: the nine windows a wave pulls from,
// window k being the segment's lanes moved by (ry, rz) rows and planes with
// k = (ry + 1) * 3 + (rz + 1) (k = 4 is the segment itself).  Lane l lies at
// x = x0 + l, or at x = l - brk on the next row for l >= brk.
struct alignas(16) D19Rec {
    uint64_t m[9];       // simulated voxels of window k
    uint32_t pre[9];     // compact index of the first simulated voxel of that window
    uint32_t edges;      // bit 2k: the voxel at x - 1 of window k's lane 0 is simulated; bit 2k + 1:
                         // the one at x + 1 of its lane 63
    uint32_t v0;         // grid index of lane 0
    uint16_t x0;         // x of lane 0
    uint8_t brk, len;    // first lane on the next row (64: none); lanes inside the grid
    uint32_t pad;
};
static_assert(sizeof(D19Rec) == 128, "D19Rec layout");

// row of the pull source x - c_i
constexpr int ROW[kQ] = {4, 4, 4, 1, 7, 3, 5, 1, 7, 1, 7, 3, 5, 3, 5, 0, 2, 6, 8};

struct D19Args {
    const float *__restrict__ fin;
    float *__restrict__ fout;
    const D19Rec *__restrict__ rec;
    const uint32_t *__restrict__ list;  // segments holding simulated voxels
    const float *__restrict__ omega;    // compact
    const float *__restrict__ kn;       // k n, compact (reactive problem only)
    const float *__restrict__ src;      // a given source per voxel (dense), or null
    float *__restrict__ csnap;          // C at the previous measured step (compact)
    double *__restrict__ part;          // per-block partial sums (measured steps)
    int64_t nent;
    int nx, ny, nz, nblk;
    double sh0, slope;                  // shift of the stored populations
    double ab_in, ab_out;               // anti-bounce-back constants in the shifted form
    double c_in, c_out;
    int react_outlet;                   // 1: zero-gradient outlet (no open links at x = nx - 1)
    int open_inlet;                     // 1: open links at x = 0 (0 for the potential problem)
    int reverse;                        // 1: each XCD walks its eighth of the list backwards
};

// Blocks are dealt round-robin to the 8 XCDs; give XCD k the k-th contiguous
// eighth of the list instead.
__device__ __forceinline__ int64_t xcd_block(int b, int nblk) {
    if (nblk < 8) return b;
    const int q = nblk >> 3, r = nblk & 7, x = b & 7;
    return (int64_t)x * q + min(x, r) + (b >> 3);
}

// The same with each XCD walking its eighth backwards.  Steps alternate between
// the two, so a step starts on the rows the previous step wrote last, still in the
// XCD's L2 and the last-level cache.
__device__ __forceinline__ int64_t xcd_block_reversed(int b, int nblk) {
    if (nblk < 8) return nblk - 1 - b;
    const int q = nblk >> 3, r = nblk & 7, x = b & 7, len = q + (x < r ? 1 : 0);
    return (int64_t)x * q + min(x, r) + (len - 1 - (b >> 3));
}

// position of population i of compact voxel j in a lattice
__host__ __device__ __forceinline__ int64_t fidx(int i, int64_t j) { return (j >> 6) * (kQ * 64) + i * 64 + (j & 63); }

// the same as a byte offset in 32 bits (a lattice is kept below 4 GiB), so that
// loads and stores take the uniform base plus one 32-bit lane offset
__device__ __forceinline__ uint32_t fbyte(int i, uint32_t j) {
    return ((j >> 6) * (kQ * 64) + (uint32_t)i * 64 + (j & 63)) * 4u;
}

__device__ __forceinline__ float ld(const float *base, uint32_t byte) {
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(base) + byte);
}

__device__ __forceinline__ void st(float *base, uint32_t byte, float val) {
    *reinterpret_cast<float *>(reinterpret_cast<char *>(base) + byte) = val;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ uint32_t mbcnt64(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ bool bit64(uint64_t m, int l) { return ((m >> l) & 1ull) != 0; }

// One step of Eq. (21) in pull form for the segments of the list, one wave each:
// gather the post-collision populations of the previous step (half-way
// bounce-back, anti-bounce-back at open face links, periodic y and z), relax
// toward a_i C with the sink a_i S, store.  A face link is open when the voxel of
// the face plane it passes (the source row's voxel at that face) is simulated.
// MEASURE also sums the fluxes of the links just crossed and the C, k n C of the
// new state.
template <bool REACT, bool MEASURE>
__global__ __launch_bounds__(kBlock) void k_d3q19(D19Args a) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // lb: the logical block, which also indexes the partial sums, so that a measured
    // step sums the same blocks in the same order in either direction
    const int64_t lb = a.reverse ? xcd_block_reversed(blockIdx.x, a.nblk) : xcd_block(blockIdx.x, a.nblk);
    const int64_t e = lb * (kBlock / 64) + wave;
    double acc[kRed] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (e < a.nent) {
        const D19Rec &R = a.rec[a.list[e]];
        const uint64_t mown = R.m[4];
        if (bit64(mown, lane)) {
            const int x = lane < (int)R.brk ? (int)R.x0 + lane : lane - (int)R.brk;
            const uint32_t j = R.pre[4] + mbcnt64(mown);
            const double csh = a.sh0 - a.slope * x;
            // every lane loads each direction once, from its pull source or, when that
            // source is missing, its own opposite population
            float raw[kQ];
            bool have[kQ];
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                const int k = ROW[i];
                const uint64_t mr = R.m[k];
                const uint32_t c = R.pre[k] + mbcnt64(mr);
                bool fl;
                uint32_t idx;
                if (CX[i] == 0) {
                    fl = bit64(mr, lane);
                    idx = c;
                } else if (CX[i] == 1) {  // source x - 1 (none at x = 0)
                    fl = x > 0 && (lane ? bit64(mr, lane - 1) : ((R.edges >> (2 * k)) & 1u) != 0);
                    idx = c - 1u;
                } else {                  // source x + 1 (none at x = nx - 1)
                    fl = x < a.nx - 1 && (lane < 63 ? bit64(mr, lane + 1) : ((R.edges >> (2 * k + 1)) & 1u) != 0);
                    idx = c + (bit64(mr, lane) ? 1u : 0u);
                }
                have[i] = fl;
                raw[i] = ld(a.fin, fl ? fbyte(i, idx) : fbyte(OPP[i], j));
            }
            double g[kQ];
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                const double w = weight(i), r = (double)raw[i];
                bool anti = false;
                double ab = 0.0;
                if (CX[i] == 1) {
                    anti = a.open_inlet && x == 0 && bit64(R.m[ROW[i]], lane);
                    ab = a.ab_in;
                } else if (CX[i] == -1) {
                    anti = !a.react_outlet && x == a.nx - 1 && bit64(R.m[ROW[i]], lane);
                    ab = a.ab_out;
                }
                g[i] = have[i] ? r + w * CX[i] * a.slope : (anti ? -r + w * ab : r);
            }
            double sum = 0.0;
#pragma unroll
            for (int i = 0; i < kQ; ++i) sum += g[i];
            const double C = csh + sum;
            const double om = (double)a.omega[j];
            const double knv = REACT ? (double)a.kn[j] : 0.0;
            const int64_t v = (int64_t)R.v0 + lane;
            const double sv = a.src ? (double)a.src[v] : 0.0;
            const double b = (om - knv) * C - om * csh + sv;
            const double keep = 1.0 - om;
#pragma unroll
            for (int i = 0; i < kQ; ++i) st(a.fout, fbyte(i, j), (float)(keep * g[i] + weight(i) * b));
            if constexpr (MEASURE) {
#pragma unroll
                for (int i = 0; i < kQ; ++i) {
                    if (CX[i] == 0) continue;
                    const double f = g[i] + weight(i) * csh;
                    if (have[i]) acc[2] += CX[i] * f;
                    if (CX[i] == 1 && a.open_inlet && x == 0 && bit64(R.m[ROW[i]], lane))
                        acc[0] += 2.0 * f - 2.0 * weight(i) * a.c_in;
                    if (CX[i] == -1 && !a.react_outlet && x == a.nx - 1 && bit64(R.m[ROW[i]], lane))
                        acc[1] += 2.0 * weight(i) * a.c_out - 2.0 * f;
                }
                acc[3] = knv * C - sv;  // the net sink
                acc[4] = C;
                acc[5] = fabs(C - (double)a.csnap[j]);
                a.csnap[j] = (float)C;
                acc[6] = fabs(C);
                acc[7] = (C == C) ? 0.0 : 1.0;
            }
        }
    }
    if constexpr (MEASURE) {
        __shared__ double red[kBlock / 64][kRed];
#pragma unroll
        for (int k = 0; k < kRed; ++k) {
            const double sm = (k == 5 || k == 6) ? wave_max(acc[k]) : wave_sum(acc[k]);
            if (lane == 0) red[wave][k] = sm;
        }
        __syncthreads();
        if (threadIdx.x < kRed) {
            const int k = threadIdx.x;
            double sm = red[0][k];
            for (int w = 1; w < kBlock / 64; ++w) sm = (k == 5 || k == 6) ? fmax(sm, red[w][k]) : sm + red[w][k];
            a.part[lb * kRed + k] = sm;
        }
    }
}

// Fixed-order final reduction of the per-block partials (one block).
__global__ __launch_bounds__(kBlock) void k_d3q19_reduce(const double *__restrict__ part, int nblk,
                                                         double *__restrict__ out) {
    __shared__ double red[kBlock / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < kRed; ++k) {
        const bool mx = k == 5 || k == 6;
        double s = 0.0;
        for (int b = threadIdx.x; b < nblk; b += kBlock) {
            const double p = part[(int64_t)b * kRed + k];
            s = mx ? fmax(s, p) : s + p;
        }
        s = mx ? wave_max(s) : wave_sum(s);
        if (lane == 0) red[wv] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = red[0];
            for (int w = 1; w < kBlock / 64; ++w) t = mx ? fmax(t, red[w]) : t + red[w];
            out[k] = t;
        }
        __syncthreads();
    }
}

// Stored state from a dense concentration field (f_i = a_i C0, NULL: C0 = 0), and
// the snapshot C used by the first window residual.  cidx maps a voxel to its
// compact index (-1 off the simulated voxels).
__global__ __launch_bounds__(kBlock) void k_d3q19_init(float *__restrict__ f, const int32_t *__restrict__ cidx,
                                                       const float *__restrict__ c0, float *__restrict__ csnap,
                                                       int64_t N, int nx, double sh0, double slope) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= N) return;
    const int32_t j = cidx[v];
    if (j < 0) return;
    const double C = c0 ? (double)c0[v] : 0.0;
    const double csh = sh0 - slope * (double)(v % nx);
#pragma unroll
    for (int i = 0; i < kQ; ++i) f[fidx(i, j)] = (float)(weight(i) * (C - csh));
    csnap[j] = (float)C;
}

// Unshifted FP64 populations of the stored (post-collision) state, dense.
__global__ __launch_bounds__(kBlock) void k_d3q19_unshift(const float *__restrict__ f, const int32_t *__restrict__ cidx,
                                                          double *__restrict__ out, int64_t N, int nx, double sh0,
                                                          double slope) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= N) return;
    const int32_t j = cidx[v];
    const double csh = sh0 - slope * (double)(v % nx);
#pragma unroll
    for (int i = 0; i < kQ; ++i) out[(int64_t)i * N + v] = j >= 0 ? (double)f[fidx(i, j)] + weight(i) * csh : 0.0;
}

// C of the state, dense: the stored populations sum to (1 - k n) C + S after the collision.
__global__ __launch_bounds__(kBlock) void k_d3q19_conc(const float *__restrict__ f, const int32_t *__restrict__ cidx,
                                                       const float *__restrict__ kn, const float *__restrict__ src,
                                                       float *__restrict__ c, int64_t N, int nx, double sh0,
                                                       double slope) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= N) return;
    const int32_t j = cidx[v];
    if (j < 0) {
        c[v] = 0.f;
        return;
    }
    double s = sh0 - slope * (double)(v % nx);
#pragma unroll
    for (int i = 0; i < kQ; ++i) s += (double)f[fidx(i, j)];
    if (src) s -= (double)src[v];
    c[v] = (float)(kn ? s / (1.0 - (double)kn[j]) : s);
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

__host__ __device__ inline int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

}  // namespace

struct lbm19_solver {
    cl::Prepared P;
    bool react = false;
    bool potential = false;        // the coupled potential problem (Dirichlet at x = L only)
    const float *src = nullptr;    // a given per-voxel source (device, dense), or null
    int64_t N = 0;                 // voxels of the simulated grid
    int64_t nf = 0, stride = 0;    // simulated voxels, and that count rounded up to 64
    int64_t nent = 0;              // segments holding simulated voxels
    int nblk = 0, nbd = 0;         // step blocks (four segments each), dense blocks
    double d0_lat = 0, ab_in = 0, ab_out = 0;
    std::vector<uint32_t> mask;    // dense per-voxel bits (pull sources, open links), for the potential solve
    std::vector<int32_t> cidx;     // dense voxel -> compact index, -1 off the simulated voxels
    std::vector<D19Rec> rec;       // per row segment
    std::vector<uint32_t> list;    // segments holding simulated voxels
    std::vector<float> om_c, kn_c; // compact 1/tau and k n
    // workspace carve-up
    size_t off_f[2] = {0, 0}, off_mask = 0, off_cidx = 0, off_rec = 0, off_list = 0, off_om = 0, off_kn = 0,
           off_cs = 0, off_part = 0, off_red = 0, need = 0;
    char *ws = nullptr;
    hipStream_t st = nullptr;
    int device = 0;
    int cur = 0;
    int64_t steps = 0;
    int measured = 0;
    lbm_run_info last{};
    double red[kRed] = {};

    template <class T>
    T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }

    D19Args args(bool measure) {
        D19Args a{};
        a.fin = at<float>(off_f[cur]);
        a.fout = at<float>(off_f[cur ^ 1]);
        a.rec = at<D19Rec>(off_rec);
        a.list = at<uint32_t>(off_list);
        a.omega = at<float>(off_om);
        a.kn = react ? at<float>(off_kn) : nullptr;
        a.src = src;
        a.csnap = at<float>(off_cs);
        a.part = measure ? at<double>(off_part) : nullptr;
        a.nent = nent;
        a.nx = P.nx;
        a.ny = P.ny;
        a.nz = P.nz;
        a.nblk = nblk;
        a.sh0 = P.sh0;
        a.slope = P.slope;
        a.ab_in = ab_in;
        a.ab_out = ab_out;
        a.c_in = P.params.c_in;
        a.c_out = P.params.c_out;
        a.react_outlet = react ? 1 : 0;
        a.open_inlet = potential ? 0 : 1;
        a.reverse = (int)(steps & 1);
        return a;
    }

    hipError_t launch(bool measure) {
        const D19Args a = args(measure);
        if (nblk > 0) {
            if (react) {
                if (measure)
                    k_d3q19<true, true><<<nblk, kBlock, 0, st>>>(a);
                else
                    k_d3q19<true, false><<<nblk, kBlock, 0, st>>>(a);
            } else {
                if (measure)
                    k_d3q19<false, true><<<nblk, kBlock, 0, st>>>(a);
                else
                    k_d3q19<false, false><<<nblk, kBlock, 0, st>>>(a);
            }
        }
        hipError_t e = hipGetLastError();
        if (e == hipSuccess && measure) {
            k_d3q19_reduce<<<1, kBlock, 0, st>>>(at<double>(off_part), nblk, at<double>(off_red));
            e = hipGetLastError();
        }
        cur ^= 1;
        ++steps;
        return e;
    }

    // one measured step; fills `last` from the reduction
    int measure_step(int64_t window) {
        hipError_t e = launch(true);
        if (e == hipSuccess) e = hipMemcpyAsync(red, at<double>(off_red), sizeof(red), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return cl::record_error(e, "lbm19 measure");
        const double A = (double)P.ny * P.nz;
        last.steps = steps;
        last.j_in = red[0] / A;
        last.j_out = red[1] / A;
        last.j_vol = P.nx > 1 ? red[2] / (P.nx - 1) / A : red[0] / A;
        last.rate = red[3] / A;
        last.mass = red[4];
        last.residual = red[6] > 0 ? red[5] / ((double)std::max<int64_t>(window, 1) * red[6]) : 0.0;
        measured = 1;
        if (red[7] != 0.0 || !std::isfinite(red[4])) return LBM_ERR_DIVERGED;
        return LBM_OK;
    }
};

// The solver behind lbm19_create; `potential` builds the coupled potential
// problem instead: transport on ionomer joined to the membrane face x = L,
// Dirichlet there, zero flux at x = 0 (the caller passes a proton-mode problem
// with c_in = c_out = the membrane potential).
static int create19(const lbm_grid *g, const uint8_t *phase, const lbm_params *p, bool potential,
                    lbm19_solver **out) {
    try {
        if (!g || !phase || !p || !out) return LBM_ERR_INVALID_ARG;
        *out = nullptr;
        auto s = std::make_unique<lbm19_solver>();
        const int st = cl::prepare(*g, phase, *p, s->P);
        if (st != LBM_OK) return st;
        cl::Prepared &P = s->P;
        if ((int64_t)kQ * P.nx * P.ny * P.nz > ((int64_t)1 << 40)) return LBM_ERR_INVALID_ARG;
        s->react = P.mode == LBM_MODE_REACT;
        s->potential = potential;
        if (potential) {
            // ionomer joined to the membrane face through ionomer (breadth-first, periodic y, z)
            const int nx = P.nx, ny = P.ny, nz = P.nz;
            const int64_t Nv = (int64_t)nx * ny * nz;
            std::vector<uint8_t> reach(Nv, 0);
            std::vector<int64_t> queue;
            for (int z = 0; z < nz; ++z)
                for (int y = 0; y < ny; ++y) {
                    const int64_t v = ((int64_t)z * ny + y) * nx + nx - 1;
                    if (P.phase[v] == LBM_IONOMER) {
                        reach[v] = 1;
                        queue.push_back(v);
                    }
                }
            for (size_t h = 0; h < queue.size(); ++h) {
                const int64_t v = queue[h];
                const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((int64_t)nx * ny));
                const int64_t nb[6] = {x > 0 ? v - 1 : -1, x + 1 < nx ? v + 1 : -1,
                                       ((int64_t)z * ny + wrapi(y - 1, ny)) * nx + x,
                                       ((int64_t)z * ny + wrapi(y + 1, ny)) * nx + x,
                                       ((int64_t)wrapi(z - 1, nz) * ny + y) * nx + x,
                                       ((int64_t)wrapi(z + 1, nz) * ny + y) * nx + x};
                for (int64_t u : nb)
                    if (u >= 0 && !reach[u] && P.phase[u] == LBM_IONOMER) {
                        reach[u] = 1;
                        queue.push_back(u);
                    }
            }
            P.percolates = false;
            for (int64_t v = 0; v < Nv; ++v) {
                if (!reach[v]) P.omega_dense[v] = 0.f;
                else P.percolates = true;
                P.active[v] = reach[v];
            }
        }
        s->N = (int64_t)P.nx * P.ny * P.nz;
        s->nbd = (int)((s->N + kBlock - 1) / kBlock);
        s->d0_lat = (P.params.tau_ref - 0.5) * P.d0 / (3.0 * P.d_ref);
        s->ab_in = 2.0 * (P.params.c_in - P.sh0);
        s->ab_out = 2.0 * (P.params.c_out - (P.sh0 - P.slope * (P.nx - 1)));
        const int nx = P.nx, ny = P.ny, nz = P.nz;
        // dense bits: missing pull sources, open face links, simulated (the potential solve reads them)
        s->mask.assign(s->N, 0u);
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const int64_t v = ((int64_t)z * ny + y) * nx + x;
                    if (!P.active[v]) continue;
                    uint32_t m = kActive;
                    for (int i = 0; i < kQ; ++i) {
                        const int sx = x - CX[i], sy = wrapi(y - CY[i], ny), sz = wrapi(z - CZ[i], nz);
                        const int64_t plane = ((int64_t)sz * ny + sy) * nx;
                        if (sx < 0 || sx >= nx || !P.active[plane + sx]) m |= 1u << i;
                        // a face link is open when the boundary-plane voxel it passes is simulated
                        if (CX[i] == 1 && x == 0 && !potential && P.active[plane]) m |= 1u << (19 + FACE_SLOT[i]);
                        if (CX[i] == -1 && x == nx - 1 && !s->react && P.active[plane + nx - 1])
                            m |= 1u << (24 + FACE_SLOT[i]);
                    }
                    s->mask[v] = m;
                }
        // compact order (x fastest) and rank of every grid position among the simulated voxels
        s->cidx.assign(s->N, -1);
        int64_t nf = 0;
        const int64_t nw = s->N / 64 + 2;
        std::vector<uint64_t> sb(nw, 0ull);
        std::vector<int64_t> rank(nw, 0);
        for (int64_t v = 0; v < s->N; ++v)
            if (P.active[v]) {
                s->cidx[v] = (int32_t)nf++;
                sb[v >> 6] |= 1ull << (v & 63);
            }
        for (int64_t w = 1; w < nw; ++w) rank[w] = rank[w - 1] + __builtin_popcountll(sb[w - 1]);
        auto bits = [&](int64_t pos, int len) {  // simulated bits of grid indices pos .. pos + len - 1
            const int64_t w = pos >> 6;
            const int sh = (int)(pos & 63);
            uint64_t v = sb[w] >> sh;
            if (sh) v |= sb[w + 1] << (64 - sh);
            return len >= 64 ? v : v & ((1ull << len) - 1ull);
        };
        auto rank_at = [&](int64_t pos) {
            const int sh = (int)(pos & 63);
            return rank[pos >> 6] + (sh ? __builtin_popcountll(sb[pos >> 6] & ((1ull << sh) - 1ull)) : 0);
        };
        auto sim = [&](int64_t pos) { return pos >= 0 && pos < s->N && ((sb[pos >> 6] >> (pos & 63)) & 1ull); };
        s->nf = nf;
        s->stride = (nf + 63) / 64 * 64;
        // one lattice below 4 GiB: byte offsets in 32 bits
        if ((int64_t)kQ * 4 * std::max<int64_t>(s->stride, 64) >= ((int64_t)1 << 32)) return LBM_ERR_INVALID_ARG;
        if (s->N >= ((int64_t)1 << 32)) return LBM_ERR_INVALID_ARG;
        // segments: the windows of the D3Q7 layout (Prepared::win_v0, win_len)
        const int64_t nseg = (int64_t)P.win_v0.size();
        const int64_t plane = (int64_t)ny * nx;
        s->rec.assign(nseg, D19Rec{});
        s->list.clear();
        for (int64_t g = 0; g < nseg; ++g) {
            D19Rec &R = s->rec[g];
            const int64_t v0 = P.win_v0[g];
            const int len = P.win_len[g];
            const int64_t row = v0 / nx;
            const int x0 = (int)(v0 - row * nx), y = (int)(row % ny), z = (int)(row / ny);
            const int brk = x0 + len > nx ? nx - x0 : 64;
            const int x63 = 63 < brk ? x0 + 63 : 63 - brk;  // x of lane 63 when the window is full
            R.v0 = (uint32_t)v0;
            R.x0 = (uint16_t)x0;
            R.brk = (uint8_t)brk;
            R.len = (uint8_t)len;
            for (int k = 0; k < 9; ++k) {
                const int ry = k / 3 - 1, rz = k % 3 - 1;
                // one offset for every lane: windows never straddle the rows where y wraps
                const int64_t oy = ry == 0 ? 0 : (ry < 0 ? (y == 0 ? (int64_t)(ny - 1) * nx : -(int64_t)nx)
                                                         : (y == ny - 1 ? -(int64_t)(ny - 1) * nx : (int64_t)nx));
                const int64_t oz = rz == 0 ? 0 : (rz < 0 ? (z == 0 ? (int64_t)(nz - 1) * plane : -plane)
                                                         : (z == nz - 1 ? -(int64_t)(nz - 1) * plane : plane));
                const int64_t w0 = v0 + oy + oz;
                R.m[k] = bits(w0, len);
                R.pre[k] = (uint32_t)rank_at(w0);
                if (x0 > 0 && sim(w0 - 1)) R.edges |= 1u << (2 * k);
                if (len == 64 && x63 < nx - 1 && sim(w0 + 64)) R.edges |= 1u << (2 * k + 1);
            }
            if (R.m[4]) s->list.push_back((uint32_t)g);
        }
        // Walk the list as four y slabs, each plane by plane: with the XCD-aware block
        // order each XCD then steps half a slab, and the rows a segment pulls from
        // (y -+ 1, z -+ 1 and the four yz diagonals) were touched a slab plane
        // earlier, still in its L2 (4 slabs measured faster than 8 or 16 here).
        if (ny >= 8) {
            const int64_t yb = (ny + 3) / 4;
            auto key = [&](uint32_t g) {  // (slab of the window's first row, plane, grid index)
                const int64_t v0 = s->rec[g].v0, row = v0 / nx, y = row % ny, z = row / ny;
                return ((y / yb) * nz + z) * plane + (v0 - z * plane);
            };
            std::sort(s->list.begin(), s->list.end(), [&](uint32_t a, uint32_t b) { return key(a) < key(b); });
        }
        s->nent = (int64_t)s->list.size();
        s->nblk = (int)((s->nent + kBlock / 64 - 1) / (kBlock / 64));
        s->om_c.assign(std::max<int64_t>(nf, 1), 0.f);
        s->kn_c.assign(s->react ? std::max<int64_t>(nf, 1) : 0, 0.f);
        for (int64_t v = 0; v < s->N; ++v) {
            const int32_t j = s->cidx[v];
            if (j < 0) continue;
            s->om_c[j] = P.omega_dense[v];
            if (s->react && ((P.params.reactive_fluids >> P.phase[v]) & 1u))
                s->kn_c[j] = (float)(P.params.k_lat * P.n_cat[v]);
        }
        // workspace: two lattices, the dense bits and compact map, records, list,
        // 1/tau, k n, C snapshot, partials, result
        size_t o = 0;
        auto take = [&](size_t bytes) {
            const size_t r = o;
            o += align256(std::max<size_t>(bytes, 1));
            return r;
        };
        const size_t fb = sizeof(float) * kQ * (size_t)std::max<int64_t>(s->stride, 64);
        s->off_f[0] = take(fb);
        s->off_f[1] = take(fb);
        s->off_mask = take(4 * (size_t)s->N);
        s->off_cidx = take(4 * (size_t)s->N);
        s->off_rec = take(sizeof(D19Rec) * (size_t)nseg);
        s->off_list = take(4 * std::max<size_t>(s->list.size(), 1));
        s->off_om = take(4 * (size_t)std::max<int64_t>(nf, 1));
        s->off_kn = s->react ? take(4 * (size_t)std::max<int64_t>(nf, 1)) : 0;
        s->off_cs = take(4 * (size_t)std::max<int64_t>(nf, 1));
        s->off_part = take(sizeof(double) * kRed * (size_t)std::max(s->nblk, 1));
        s->off_red = take(sizeof(double) * kRed);
        s->need = o;
        *out = s.release();
        return LBM_OK;
    } catch (...) {
        return LBM_ERR_INVALID_ARG;
    }
}


namespace {

// ---- coupled oxygen / proton-potential problem (Eqs. 15-18b, Tafel Eq. 17b)

// O2 sink of each reaction site from the potential: k n = k_ref n exp(beta (phi - phi_ref))
__global__ __launch_bounds__(kBlock) void k_cpl_rate(float *__restrict__ kn_o2, const int32_t *__restrict__ cidx_o2,
                                                     const float *__restrict__ n_site, const float *__restrict__ phi,
                                                     int64_t Ns, int nx, int nx_o, int off, double k_ref, double beta,
                                                     double phi_ref) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= Ns) return;
    const int64_t row = v / nx, x = v - row * nx;
    const int32_t j = cidx_o2[row * nx_o + x + off];
    if (j < 0) return;
    const double n = (double)n_site[v];
    kn_o2[j] = n > 0.0 ? (float)(k_ref * n * exp(beta * ((double)phi[v] - phi_ref))) : 0.f;
}

// proton source of each site (Eq. 18b) from C and the potential, as the LBM source
// S = -gamma n (C / C_in) exp(beta (phi - phi_ref))
__global__ __launch_bounds__(kBlock) void k_cpl_source(float *__restrict__ src, const float *__restrict__ n_site,
                                                       const float *__restrict__ phi, const float *__restrict__ c_o2,
                                                       int64_t Ns, int nx, int nx_o, int off, double gamma,
                                                       double beta, double phi_ref, double c_in) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= Ns) return;
    const int64_t row = v / nx, x = v - row * nx;
    const double n = (double)n_site[v];
    const double C = (double)c_o2[row * nx_o + x + off];
    src[v] = n > 0.0 ? (float)(-gamma * n * (C / c_in) * exp(beta * ((double)phi[v] - phi_ref))) : 0.f;
}

// phi <- phi + theta (phi_solved - phi) on the potential's voxels (phi_m elsewhere);
// per-block max of |phi_solved - phi| and min of the new phi
__global__ __launch_bounds__(kBlock) void k_cpl_relax(float *__restrict__ phi, const float *__restrict__ solved,
                                                      const uint32_t *__restrict__ mask, int64_t Ns, double theta,
                                                      double phi_m, float *__restrict__ part) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double d = 0.0, lo = phi_m;
    if (v < Ns) {
        const double old = (double)phi[v];
        const double nw = (mask[v] & kActive) ? (double)solved[v] : phi_m;
        d = fabs(nw - old);
        const double upd = old + theta * (nw - old);
        phi[v] = (float)upd;
        lo = upd;
    }
    d = wave_max(d);
    for (int o = 32; o > 0; o >>= 1) lo = fmin(lo, __shfl_xor(lo, o));
    __shared__ double red[2][kBlock / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wv] = d;
        red[1][wv] = lo;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = red[0][0], b = red[1][0];
        for (int w = 1; w < kBlock / 64; ++w) {
            a = fmax(a, red[0][w]);
            b = fmin(b, red[1][w]);
        }
        part[2 * (int64_t)blockIdx.x] = (float)a;
        part[2 * (int64_t)blockIdx.x + 1] = (float)b;
    }
}

__global__ __launch_bounds__(kBlock) void k_cpl_fill(float *__restrict__ a, int64_t n, float val) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v < n) a[v] = val;
}

// ---- the potential's steady state at tau_phi = 1 by preconditioned conjugate gradients
//
// With tau = 1 every post-collision population of the potential lattice is a_i u,
// u = phi + S (S the source the collision adds), so its steady state is the
// solution of the link Laplacian of the D3Q19 links (Eqs. 21-24 at tau = 1):
//   sum over links to simulated voxels  a_i (u(x) - u(x - c_i))
// + sum over open membrane-face links 2 a_i (u(x) - phi_m)            = S(x),
// symmetric positive definite on the voxels the membrane face reaches.  The
// conjugate-gradient iteration with the inverse diagonal as preconditioner solves
// it in FP64; the lattice then takes the equilibrium state a_i u, which the
// stepping would have reached.  Vectors are dense over the structure grid (zero
// off the potential's voxels); per-block partial sums, then one-block finishing
// kernels that keep the iteration's scalars on the device.
struct Pcg {
    const uint32_t *mask;
    double *u, *r, *p, *ap, *dinv, *part, *scal;  // scal: rz, alpha, beta, rmax, bmax, pap
    int64_t N;
    int nx, ny, nz, nblk;
    double phi_m;
};
enum { P_RZ = 0, P_ALPHA, P_BETA, P_RMAX, P_BMAX, P_PAP };

// per block: the sum of a, the maxima of m1 and m2 (three partial slots)
__device__ __forceinline__ void block_sums(double a, double m1, double m2, double *part) {
    __shared__ double red[3][kBlock / 64];
    a = wave_sum(a);
    m1 = wave_max(m1);
    m2 = wave_max(m2);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wv] = a;
        red[1][wv] = m1;
        red[2][wv] = m2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0.0, x1 = 0.0, x2 = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) {
            s0 += red[0][w];
            x1 = fmax(x1, red[1][w]);
            x2 = fmax(x2, red[2][w]);
        }
        part[3 * (int64_t)blockIdx.x] = s0;
        part[3 * (int64_t)blockIdx.x + 1] = x1;
        part[3 * (int64_t)blockIdx.x + 2] = x2;
    }
}

// (A q)(v) on the potential's voxels, the diagonal and the open-link sum
__device__ __forceinline__ double pcg_apply(const Pcg &g, int64_t v, const double *__restrict__ q, double &diag,
                                            double &open) {
    const uint32_t m = g.mask[v];
    const uint32_t vv = (uint32_t)v, nx = (uint32_t)g.nx, ny = (uint32_t)g.ny, r = vv / nx;
    const int x = (int)(vv - r * nx), z = (int)(r / ny), y = (int)(r - (uint32_t)z * ny);
    double off = 0.0;
    diag = 0.0;
    open = 0.0;
#pragma unroll
    for (int i = 1; i < kQ; ++i) {
        const double w = weight(i);
        if (!((m >> i) & 1u)) {
            const int sy = wrapi(y - CY[i], g.ny), sz = wrapi(z - CZ[i], g.nz);
            off += w * q[((int64_t)sz * g.ny + sy) * g.nx + (x - CX[i])];
            diag += w;
        } else if (CX[i] == -1 && x == g.nx - 1 && ((m >> (24 + FACE_SLOT[i])) & 1u)) {
            open += 2.0 * w;
        }
    }
    diag += open;
    return diag * q[v] - off;
}

// u = phi + S (the previous potential as the first guess), the inverse diagonal
__global__ __launch_bounds__(kBlock) void k_pcg_start(Pcg g, const float *__restrict__ phi,
                                                      const float *__restrict__ src) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= g.N) return;
    const bool act = (g.mask[v] & kActive) != 0;
    g.u[v] = act ? (double)phi[v] + (double)src[v] : 0.0;
    g.p[v] = 0.0;
    double d = 0.0;
    if (act) {
        const uint32_t m = g.mask[v];
        const int x = (int)(v % g.nx);
        for (int i = 1; i < kQ; ++i) {
            if (!((m >> i) & 1u)) d += weight(i);
            else if (CX[i] == -1 && x == g.nx - 1 && ((m >> (24 + FACE_SLOT[i])) & 1u)) d += 2.0 * weight(i);
        }
    }
    g.dinv[v] = d > 0.0 ? 1.0 / d : 0.0;
}

// r = b - A u, p = M^-1 r; partials of r.M^-1 r, max|r| and max|b|
__global__ __launch_bounds__(kBlock) void k_pcg_residual(Pcg g, const float *__restrict__ src) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double rz = 0.0, rm = 0.0, bm = 0.0;
    if (v < g.N) {
        double rv = 0.0;
        if (g.mask[v] & kActive) {
            double diag, open;
            const double au = pcg_apply(g, v, g.u, diag, open);
            const double b = (double)src[v] + open * g.phi_m;
            rv = b - au;
            bm = fabs(b);
        }
        g.r[v] = rv;
        const double z = g.dinv[v] * rv;
        g.p[v] = z;
        rz = rv * z;
        rm = fabs(rv);
    }
    block_sums(rz, rm, bm, g.part);
}

// ap = A p; partials of p.ap
__global__ __launch_bounds__(kBlock) void k_pcg_ap(Pcg g) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double pap = 0.0;
    if (v < g.N) {
        double a = 0.0;
        if (g.mask[v] & kActive) {
            double diag, open;
            a = pcg_apply(g, v, g.p, diag, open);
        }
        g.ap[v] = a;
        pap = g.p[v] * a;
    }
    block_sums(pap, 0.0, 0.0, g.part);
}

// one block: sums of the partials; stage 0 after the residual (rz, bmax, rmax),
// 1 after A p (alpha = rz / pap), 2 after the update (beta = rz_new / rz, rz, rmax)
__global__ __launch_bounds__(kBlock) void k_pcg_finish(Pcg g, int stage) {
    double a = 0.0, m1 = 0.0, m2 = 0.0;
    for (int k = threadIdx.x; k < g.nblk; k += kBlock) {
        a += g.part[3 * (int64_t)k];
        m1 = fmax(m1, g.part[3 * (int64_t)k + 1]);
        m2 = fmax(m2, g.part[3 * (int64_t)k + 2]);
    }
    __shared__ double red[3][kBlock / 64];
    a = wave_sum(a);
    m1 = wave_max(m1);
    m2 = wave_max(m2);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wv] = a;
        red[1][wv] = m1;
        red[2][wv] = m2;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double s0 = 0.0, x1 = 0.0, x2 = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) {  // fixed order: the scalars are deterministic
        s0 += red[0][w];
        x1 = fmax(x1, red[1][w]);
        x2 = fmax(x2, red[2][w]);
    }
    if (stage == 0) {
        g.scal[P_RZ] = s0;
        g.scal[P_RMAX] = x1;
        g.scal[P_BMAX] = x2;
    } else if (stage == 1) {
        g.scal[P_PAP] = s0;
        g.scal[P_ALPHA] = s0 > 0.0 ? g.scal[P_RZ] / s0 : 0.0;
    } else {
        g.scal[P_BETA] = g.scal[P_RZ] > 0.0 ? s0 / g.scal[P_RZ] : 0.0;
        g.scal[P_RZ] = s0;
        g.scal[P_RMAX] = x1;
    }
}

// u += alpha p, r -= alpha ap; partials of r.M^-1 r and max|r|
__global__ __launch_bounds__(kBlock) void k_pcg_update(Pcg g) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double rz = 0.0, rm = 0.0;
    if (v < g.N) {
        const double al = g.scal[P_ALPHA];
        g.u[v] += al * g.p[v];
        const double rv = g.r[v] - al * g.ap[v];
        g.r[v] = rv;
        rz = rv * g.dinv[v] * rv;
        rm = fabs(rv);
    }
    block_sums(rz, rm, 0.0, g.part);
}

// p = M^-1 r + beta p
__global__ __launch_bounds__(kBlock) void k_pcg_direction(Pcg g) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= g.N) return;
    g.p[v] = g.dinv[v] * g.r[v] + g.scal[P_BETA] * g.p[v];
}

// FP32 copy of u for the lattice's equilibrium state
__global__ __launch_bounds__(kBlock) void k_pcg_out(Pcg g, float *__restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v < g.N) out[v] = (float)g.u[v];
}

}  // namespace

struct lbm19_coupled {
    lbm19_solver *o2 = nullptr, *phi = nullptr;
    lbm_coupling cp{};
    double c_in = 1.0;
    int nx = 0, ny = 0, nz = 0, nx_o = 0, off = 0;
    int64_t Ns = 0;
    int nb = 0;
    std::vector<float> n_site;
    size_t ws_o2 = 0, ws_phi = 0, off_phi_ws = 0, off_n = 0, off_phi = 0, off_new = 0, off_c = 0, off_src = 0,
           off_part = 0, off_pcg = 0, need = 0;
    bool use_cg = false;  // the potential by conjugate gradients (tau_phi = 1)
    char *ws = nullptr;
    hipStream_t st = nullptr;
    lbm_coupled_info last{};
    template <class T>
    T *at(size_t o) const { return reinterpret_cast<T *>(ws + o); }
    ~lbm19_coupled() {
        delete o2;
        delete phi;
    }
};

extern "C" {

int lbm19_create(const lbm_grid *g, const uint8_t *phase, const lbm_params *p, lbm19_solver **out) {
    return create19(g, phase, p, false, out);
}

int lbm19_get_info(const lbm19_solver *s, lbm_info *info) {
    if (!s || !info) return LBM_ERR_INVALID_ARG;
    std::memset(info, 0, sizeof(*info));
    const cl::Prepared &P = s->P;
    info->nx = P.nx;
    info->ny = P.ny;
    info->nz = P.nz;
    info->nx_struct = P.nx_struct;
    int64_t n = 0;
    for (uint8_t a : P.active) n += a ? 1 : 0;
    info->n_active = n;
    info->n_segments = 0;
    info->d0 = P.d0;
    info->d_ref = P.d_ref;
    info->d0_lat = s->d0_lat;
    info->percolates = P.percolates ? 1 : 0;
    info->mode = P.mode;
    return LBM_OK;
}

int lbm19_workspace_bytes(const lbm19_solver *s, size_t *bytes) {
    if (!s || !bytes) return LBM_ERR_INVALID_ARG;
    *bytes = s->need;
    return LBM_OK;
}

int lbm19_bind(lbm19_solver *s, void *ws, size_t bytes, void *stream) {
    if (!s || !ws || (reinterpret_cast<uintptr_t>(ws) & 255u)) return LBM_ERR_WORKSPACE;
    if (bytes < s->need) return LBM_ERR_WORKSPACE;
    s->ws = static_cast<char *>(ws);
    s->st = static_cast<hipStream_t>(stream);
    hipError_t e = hipGetDevice(&s->device);
    auto up = [&](size_t off, const void *src, size_t n) {
        if (e == hipSuccess && n) e = hipMemcpyAsync(s->ws + off, src, n, hipMemcpyHostToDevice, s->st);
    };
    up(s->off_mask, s->mask.data(), 4 * s->mask.size());
    up(s->off_cidx, s->cidx.data(), 4 * s->cidx.size());
    up(s->off_rec, s->rec.data(), sizeof(D19Rec) * s->rec.size());
    up(s->off_list, s->list.data(), 4 * s->list.size());
    up(s->off_om, s->om_c.data(), 4 * s->om_c.size());
    if (s->react) up(s->off_kn, s->kn_c.data(), 4 * s->kn_c.size());
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) {
        s->ws = nullptr;
        return cl::record_error(e, "lbm19_bind");
    }
    return lbm19_set_initial_concentration(s, nullptr);
}

int lbm19_set_initial_concentration(lbm19_solver *s, const float *c_dev) {
    if (!s) return LBM_ERR_INVALID_ARG;
    if (!s->ws) return LBM_ERR_UNBOUND;
    s->cur = 0;
    k_d3q19_init<<<s->nbd, kBlock, 0, s->st>>>(s->at<float>(s->off_f[0]), s->at<int32_t>(s->off_cidx), c_dev,
                                               s->at<float>(s->off_cs), s->N, s->P.nx, s->P.sh0, s->P.slope);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    s->steps = 0;
    s->measured = 0;
    std::memset(&s->last, 0, sizeof(s->last));
    return e == hipSuccess ? LBM_OK : cl::record_error(e, "lbm19_set_initial_concentration");
}

int lbm19_step(lbm19_solver *s, int64_t nsteps) {
    if (!s || nsteps < 0) return LBM_ERR_INVALID_ARG;
    if (!s->ws) return LBM_ERR_UNBOUND;
    for (int64_t k = 0; k < nsteps; ++k) {
        const hipError_t e = s->launch(false);
        if (e != hipSuccess) return cl::record_error(e, "lbm19_step");
    }
    return LBM_OK;
}

int lbm19_measure(lbm19_solver *s, lbm_run_info *info) {
    if (!s) return LBM_ERR_INVALID_ARG;
    if (!s->ws) return LBM_ERR_UNBOUND;
    const int st = s->measure_step(1);
    s->last.status = st;
    if (info) *info = s->last;
    return st;
}

int lbm19_run_to_steady(lbm19_solver *s, lbm_run_info *info) {
    if (!s) return LBM_ERR_INVALID_ARG;
    if (!s->ws) return LBM_ERR_UNBOUND;
    const lbm_params &p = s->P.params;
    if (!s->react && !s->P.percolates) {
        s->last.status = LBM_ERR_NO_PERCOLATION;
        if (info) *info = s->last;
        return LBM_ERR_NO_PERCOLATION;
    }
    const int64_t K = std::max<int64_t>(2, p.check_every);
    // Stop when, over windows of K steps, (i) the C field moves by less than
    // tol_change per step relative to max C, (ii) the output (mean interior flux,
    // the total sink when reacting, the membrane current of the potential
    // problem) is within tol_flux of its limit, estimated
    // from the ratio rho of successive window changes as |d| max(1, rho/(1-rho)),
    // on two checks in a row, and (iii) the balance J_in - J_out - R (R the net
    // sink) closes to tol_balance of the largest of the three.
    double q[3] = {0, 0, 0};
    int nq = 0, good = 0, st = LBM_NOT_CONVERGED;
    s->last.checks = 0;
    while (s->steps < p.max_steps) {
        const int64_t w = std::min<int64_t>(K, p.max_steps - s->steps);
        int rc = lbm19_step(s, w - 1);
        if (rc == LBM_OK) rc = s->measure_step(w);
        if (rc != LBM_OK) {
            st = rc;
            break;
        }
        ++s->last.checks;
        const double qk = s->react ? s->last.rate : (s->potential ? s->last.j_out : s->last.j_vol);
        q[0] = q[1];
        q[1] = q[2];
        q[2] = qk;
        nq = std::min(nq + 1, 3);
        double est = INFINITY;
        if (nq == 3 && qk != 0.0) {
            const double d1 = q[2] - q[1], d0 = q[1] - q[0];
            const double rho = d0 != 0.0 ? d1 / d0 : 0.0;
            if (rho < 1.0) est = std::fabs(d1) / std::fabs(qk) * std::max(1.0, rho > 0 ? rho / (1.0 - rho) : 0.0);
        }
        s->last.est_error = est;
        const double den = std::max({std::fabs(s->last.j_in), std::fabs(s->last.j_out), std::fabs(s->last.rate)});
        const double bal = den > 0.0 ? std::fabs(s->last.j_in - s->last.j_out - s->last.rate) / den : INFINITY;
        const bool ok = s->last.residual < p.tol_change && est < p.tol_flux && bal < p.tol_balance;
        good = ok ? good + 1 : 0;
        if (good >= 2) {
            st = LBM_OK;
            break;
        }
    }
    s->last.status = st;
    if (info) *info = s->last;
    return st;
}

int lbm19_deff(const lbm19_solver *s, double *out) {
    if (!s || !out) return LBM_ERR_INVALID_ARG;
    if (s->react) return LBM_ERR_WRONG_MODE;
    if (!s->P.percolates) {
        *out = 0.0;
        return LBM_ERR_NO_PERCOLATION;
    }
    if (!s->measured) return LBM_ERR_UNBOUND;
    const double dc = s->P.params.c_in - s->P.params.c_out;
    if (dc == 0.0) return LBM_ERR_INVALID_ARG;
    *out = s->last.j_vol * s->P.nx / (dc * s->d0_lat);
    return s->last.status == LBM_NOT_CONVERGED ? LBM_NOT_CONVERGED : LBM_OK;
}

int lbm19_reaction_rate(const lbm19_solver *s, double *rate, double *jin) {
    if (!s) return LBM_ERR_INVALID_ARG;
    if (!s->react) return LBM_ERR_WRONG_MODE;
    if (!s->measured) return LBM_ERR_UNBOUND;
    if (rate) *rate = s->last.rate;
    if (jin) *jin = s->last.j_in;
    return s->last.status == LBM_NOT_CONVERGED ? LBM_NOT_CONVERGED : LBM_OK;
}

int lbm19_get_populations(const lbm19_solver *s, double *f_dev) {
    if (!s || !f_dev) return LBM_ERR_INVALID_ARG;
    if (!s->ws) return LBM_ERR_UNBOUND;
    k_d3q19_unshift<<<s->nbd, kBlock, 0, s->st>>>(s->at<float>(s->off_f[s->cur]), s->at<int32_t>(s->off_cidx), f_dev,
                                                  s->N, s->P.nx, s->P.sh0, s->P.slope);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    return e == hipSuccess ? LBM_OK : cl::record_error(e, "lbm19_get_populations");
}

int lbm19_concentration(const lbm19_solver *s, float *c_dev) {
    if (!s || !c_dev) return LBM_ERR_INVALID_ARG;
    if (!s->ws) return LBM_ERR_UNBOUND;
    k_d3q19_conc<<<s->nbd, kBlock, 0, s->st>>>(s->at<float>(s->off_f[s->cur]), s->at<int32_t>(s->off_cidx),
                                               s->react ? s->at<float>(s->off_kn) : nullptr, s->src, c_dev, s->N,
                                               s->P.nx, s->P.sh0, s->P.slope);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    return e == hipSuccess ? LBM_OK : cl::record_error(e, "lbm19_concentration");
}

void lbm19_destroy(lbm19_solver *s) { delete s; }


int lbm_coupling_default(lbm_coupling *c) {
    if (!c) return LBM_ERR_INVALID_ARG;
    std::memset(c, 0, sizeof(*c));
    c->struct_size = sizeof(lbm_coupling);
    c->k_ref = 1e-2;
    c->beta = 21.3;
    c->gamma = 1e-3;
    c->phi_m = 0.6;
    c->phi_ref = 0.6;
    c->tau_phi = 1.0;
    c->theta = 0.5;
    c->tol_phi = 1e-6;
    c->max_iter = 200;
    return LBM_OK;
}

int lbm19_coupled_create(const lbm_grid *g, const uint8_t *phase, const lbm_params *p, const lbm_coupling *cp,
                         lbm19_coupled **out) {
    try {
        if (!g || !phase || !p || !cp || !out) return LBM_ERR_INVALID_ARG;
        *out = nullptr;
        if (cp->struct_size != sizeof(lbm_coupling) || !(cp->k_ref > 0.0) || !(cp->beta >= 0.0) ||
            !(cp->gamma >= 0.0) || !(cp->tau_phi > 0.5) || !(cp->theta > 0.0 && cp->theta <= 1.0) ||
            !(cp->tol_phi > 0.0) || cp->max_iter < 1 || p->mode != LBM_MODE_REACT || !(p->c_in > 0.0) ||
            cp->potential_solver < 0 || cp->potential_solver > 1)
            return LBM_ERR_INVALID_ARG;
        // the largest site rate, at the membrane potential, must keep k n below 1
        if (6.0 * cp->k_ref * std::exp(cp->beta * std::max(0.0, cp->phi_m - cp->phi_ref)) >= 1.0)
            return LBM_ERR_UNSTABLE;
        auto c = std::make_unique<lbm19_coupled>();
        c->cp = *cp;
        c->c_in = p->c_in;
        lbm_params po = *p;
        po.k_lat = cp->k_ref;
        po.catalyst_phases = 1u << LBM_PT;
        po.reactive_fluids = 1u << LBM_IONOMER;
        int st = create19(g, phase, &po, false, &c->o2);
        if (st != LBM_OK) return st;
        lbm_params pp = *p;
        pp.mode = LBM_MODE_PROTON;
        pp.c_in = pp.c_out = cp->phi_m;
        pp.tau_ref = cp->tau_phi;
        pp.knudsen = 0;
        pp.k_lat = 0.0;
        st = create19(g, phase, &pp, true, &c->phi);
        if (st != LBM_OK) return st;
        const cl::Prepared &O = c->o2->P, &F = c->phi->P;
        c->nx = F.nx;
        c->ny = F.ny;
        c->nz = F.nz;
        c->nx_o = O.nx;
        c->off = O.nx - F.nx;
        c->Ns = (int64_t)F.nx * F.ny * F.nz;
        c->nb = (int)((c->Ns + kBlock - 1) / kBlock);
        // sites: ionomer with Pt face neighbours, reached by both problems
        c->n_site.assign(c->Ns, 0.f);
        for (int64_t r = 0; r < (int64_t)F.ny * F.nz; ++r)
            for (int x = 0; x < F.nx; ++x) {
                const int64_t v = r * F.nx + x, vo = r * O.nx + x + c->off;
                if (F.active[v] && O.active[vo] && O.phase[vo] == LBM_IONOMER && O.n_cat[vo] > 0)
                    c->n_site[v] = (float)O.n_cat[vo];
            }
        // no site reached by both oxygen and protons: nothing to couple
        if (std::none_of(c->n_site.begin(), c->n_site.end(), [](float n) { return n > 0.f; }))
            return LBM_ERR_NO_PERCOLATION;
        lbm19_workspace_bytes(c->o2, &c->ws_o2);
        lbm19_workspace_bytes(c->phi, &c->ws_phi);
        size_t o = align256(c->ws_o2);
        c->off_phi_ws = o;
        o += align256(c->ws_phi);
        const size_t s4 = align256(4 * (size_t)c->Ns);
        c->off_n = o;
        o += s4;
        c->off_phi = o;
        o += s4;
        c->off_new = o;
        o += s4;
        c->off_src = o;
        o += s4;
        c->off_c = o;
        o += align256(4 * (size_t)O.nx * O.ny * O.nz);
        c->off_part = o;
        o += align256(8 * (size_t)c->nb);
        c->use_cg = cp->tau_phi == 1.0 && cp->potential_solver == 0;
        c->off_pcg = o;
        if (c->use_cg) o += 5 * align256(8 * (size_t)c->Ns) + align256(8 * 3 * (size_t)c->nb) + 256;
        c->need = o;
        *out = c.release();
        return LBM_OK;
    } catch (...) {
        return LBM_ERR_INVALID_ARG;
    }
}

int lbm19_coupled_workspace_bytes(const lbm19_coupled *c, size_t *bytes) {
    if (!c || !bytes) return LBM_ERR_INVALID_ARG;
    *bytes = c->need;
    return LBM_OK;
}

int lbm19_coupled_bind(lbm19_coupled *c, void *ws, size_t bytes, void *stream) {
    if (!c || !ws || (reinterpret_cast<uintptr_t>(ws) & 255u) || bytes < c->need) return LBM_ERR_WORKSPACE;
    c->ws = static_cast<char *>(ws);
    c->st = static_cast<hipStream_t>(stream);
    int st = lbm19_bind(c->o2, c->ws, c->ws_o2, stream);
    if (st == LBM_OK) st = lbm19_bind(c->phi, c->ws + c->off_phi_ws, c->ws_phi, stream);
    if (st != LBM_OK) {
        c->ws = nullptr;
        return st;
    }
    c->phi->src = c->at<float>(c->off_src);
    hipError_t e = hipMemcpyAsync(c->at<float>(c->off_n), c->n_site.data(), 4 * (size_t)c->Ns,
                                  hipMemcpyHostToDevice, c->st);
    if (e == hipSuccess) {
        k_cpl_fill<<<c->nb, kBlock, 0, c->st>>>(c->at<float>(c->off_phi), c->Ns, (float)c->cp.phi_m);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        k_cpl_fill<<<c->nb, kBlock, 0, c->st>>>(c->at<float>(c->off_src), c->Ns, 0.f);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e != hipSuccess) {
        c->ws = nullptr;
        return cl::record_error(e, "lbm19_coupled_bind");
    }
    // the potential starts from the membrane value everywhere
    return lbm19_set_initial_concentration(c->phi, c->at<float>(c->off_phi));
}

// The potential's steady state for the current source by preconditioned conjugate
// gradients (tau_phi = 1, see Pcg), then the lattice set to its equilibrium state
// and one measured step (fluxes and source as the stepping solver reports them).
static int potential_cg(lbm19_coupled *c, lbm_run_info *r, int64_t *iters) {
    const int64_t Ns = c->Ns;
    const size_t v8 = align256(8 * (size_t)Ns);
    Pcg g{};
    g.mask = c->phi->at<uint32_t>(c->phi->off_mask);
    g.u = c->at<double>(c->off_pcg);
    g.r = c->at<double>(c->off_pcg + v8);
    g.p = c->at<double>(c->off_pcg + 2 * v8);
    g.ap = c->at<double>(c->off_pcg + 3 * v8);
    g.dinv = c->at<double>(c->off_pcg + 4 * v8);
    g.part = c->at<double>(c->off_pcg + 5 * v8);
    g.scal = c->at<double>(c->off_pcg + 5 * v8 + align256(8 * 3 * (size_t)c->nb));
    g.N = Ns;
    g.nx = c->nx;
    g.ny = c->ny;
    g.nz = c->nz;
    g.nblk = c->nb;
    g.phi_m = c->cp.phi_m;
    const float *src = c->at<float>(c->off_src);
    hipStream_t st = c->st;
    k_pcg_start<<<c->nb, kBlock, 0, st>>>(g, c->at<float>(c->off_phi), src);
    k_pcg_residual<<<c->nb, kBlock, 0, st>>>(g, src);
    k_pcg_finish<<<1, kBlock, 0, st>>>(g, 0);
    hipError_t e = hipGetLastError();
    double sc[8] = {};
    constexpr double kTol = 1e-12;         // max|r| <= kTol max|b|
    const int64_t max_it = 200000;
    int64_t it = 0;
    bool done = false;
    while (e == hipSuccess && !done) {
        e = hipMemcpyAsync(sc, g.scal, sizeof(sc), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) break;
        if (!(sc[P_RMAX] > kTol * sc[P_BMAX]) || it >= max_it) {
            done = true;
            break;
        }
        for (int k = 0; k < 32 && e == hipSuccess; ++k, ++it) {
            k_pcg_ap<<<c->nb, kBlock, 0, st>>>(g);
            k_pcg_finish<<<1, kBlock, 0, st>>>(g, 1);
            k_pcg_update<<<c->nb, kBlock, 0, st>>>(g);
            k_pcg_finish<<<1, kBlock, 0, st>>>(g, 2);
            k_pcg_direction<<<c->nb, kBlock, 0, st>>>(g);
            e = hipGetLastError();
        }
    }
    *iters = it;
    if (e != hipSuccess) return cl::record_error(e, "lbm19_coupled_run (potential)");
    if (!(sc[P_RMAX] <= kTol * sc[P_BMAX])) return std::isfinite(sc[P_RMAX]) ? LBM_NOT_CONVERGED : LBM_ERR_DIVERGED;
    k_pcg_out<<<c->nb, kBlock, 0, st>>>(g, c->at<float>(c->off_new));
    e = hipGetLastError();
    if (e != hipSuccess) return cl::record_error(e, "lbm19_coupled_run (potential)");
    int s = lbm19_set_initial_concentration(c->phi, c->at<float>(c->off_new));
    if (s == LBM_OK) s = lbm19_measure(c->phi, r);
    return s;
}

int lbm19_coupled_run(lbm19_coupled *c, lbm_coupled_info *info) {
    if (!c) return LBM_ERR_INVALID_ARG;
    if (!c->ws) return LBM_ERR_UNBOUND;
    const lbm_coupling &cp = c->cp;
    lbm_coupled_info &I = c->last;
    std::memset(&I, 0, sizeof(I));
    I.status = LBM_NOT_CONVERGED;
    std::vector<float> part(2 * (size_t)c->nb);
    lbm_run_info r{};
    int inner = LBM_OK;
    for (int it = 1; it <= cp.max_iter; ++it) {
        // O2 with the Tafel rate of the current potential
        k_cpl_rate<<<c->nb, kBlock, 0, c->st>>>(c->o2->at<float>(c->o2->off_kn), c->o2->at<int32_t>(c->o2->off_cidx),
                                                c->at<float>(c->off_n),
                                                c->at<float>(c->off_phi), c->Ns, c->nx, c->nx_o, c->off, cp.k_ref,
                                                cp.beta, cp.phi_ref);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return cl::record_error(e, "lbm19_coupled_run");
        int st = lbm19_run_to_steady(c->o2, &r);
        I.o2_steps = r.steps;
        if (st != LBM_OK) {  // an error, or an inner solve out of steps
            inner = st;
            break;
        }
        I.rate = r.rate;
        st = lbm19_concentration(c->o2, c->at<float>(c->off_c));
        if (st < 0) return I.status = st;
        // the potential with the proton source of that O2 field
        k_cpl_source<<<c->nb, kBlock, 0, c->st>>>(c->at<float>(c->off_src), c->at<float>(c->off_n),
                                                  c->at<float>(c->off_phi), c->at<float>(c->off_c), c->Ns, c->nx,
                                                  c->nx_o, c->off, cp.gamma, cp.beta, cp.phi_ref, c->c_in);
        e = hipGetLastError();
        if (e != hipSuccess) return cl::record_error(e, "lbm19_coupled_run");
        if (c->use_cg) {
            int64_t iters = 0;
            st = potential_cg(c, &r, &iters);
            I.phi_cg_iterations += iters;
        } else {
            st = lbm19_run_to_steady(c->phi, &r);
            I.phi_steps = r.steps;
        }
        if (st != LBM_OK) {
            inner = st;
            break;
        }
        I.proton_in = -r.j_out;
        I.source = r.rate;
        st = lbm19_concentration(c->phi, c->at<float>(c->off_new));
        if (st < 0) return I.status = st;
        k_cpl_relax<<<c->nb, kBlock, 0, c->st>>>(c->at<float>(c->off_phi), c->at<float>(c->off_new),
                                                 c->phi->at<uint32_t>(c->phi->off_mask), c->Ns, cp.theta, cp.phi_m,
                                                 c->at<float>(c->off_part));
        e = hipGetLastError();
        if (e == hipSuccess)
            e = hipMemcpyAsync(part.data(), c->at<float>(c->off_part), 4 * part.size(), hipMemcpyDeviceToHost, c->st);
        if (e == hipSuccess) e = hipStreamSynchronize(c->st);
        if (e != hipSuccess) return cl::record_error(e, "lbm19_coupled_run");
        double d = 0.0, lo = cp.phi_m;
        for (int b = 0; b < c->nb; ++b) {
            d = std::max(d, (double)part[2 * (size_t)b]);
            lo = std::min(lo, (double)part[2 * (size_t)b + 1]);
        }
        I.iterations = it;
        I.dphi = d;
        I.status = LBM_NOT_CONVERGED;
        I.phi_min = lo;
        if (d < cp.tol_phi) {
            I.status = LBM_OK;
            break;
        }
    }
    if (inner != LBM_OK) I.status = inner < 0 ? inner : LBM_NOT_CONVERGED;
    if (info) *info = I;
    return I.status;
}

int lbm19_coupled_fields(const lbm19_coupled *c, float *c_dev, float *phi_dev) {
    if (!c) return LBM_ERR_INVALID_ARG;
    if (!c->ws) return LBM_ERR_UNBOUND;
    hipError_t e = hipSuccess;
    if (c_dev) {
        const int st = lbm19_concentration(c->o2, c_dev);
        if (st != LBM_OK) return st;
    }
    if (phi_dev) {
        e = hipMemcpyAsync(phi_dev, c->at<float>(c->off_phi), 4 * (size_t)c->Ns, hipMemcpyDeviceToDevice, c->st);
        if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    }
    return e == hipSuccess ? LBM_OK : cl::record_error(e, "lbm19_coupled_fields");
}

void lbm19_coupled_destroy(lbm19_coupled *c) { delete c; }

}  // extern "C"
