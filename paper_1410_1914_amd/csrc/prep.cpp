// Host preprocessing: structure -> simulated grid, local relaxation rates, sink
// coefficients and the 64-voxel segment bitmasks of the device layout.
//
// Physics follows Chen et al., arXiv 1410.1914: Section 2.1.3 (13-direction pore
// size), Section 3.1 Eqs. (7)-(9) (bulk, Knudsen, Bosanquet), Section 3.2 Eq. (15)
// (one continuous field over pore + ionomer), Section 3.3 (proton conduction in the
// ionomer), Section 3.4 Eq. (18a) (catalyst face neighbours), Section 3.5 (boundary
// problems, reservoir plane) and Section 4 Eq. (24) (tau from D).
#include "prep.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>

namespace cl {

int record_error(hipError_t e, const char *where);  // the engine's error record (lbm_last_error)

namespace {

constexpr double kR = 8.314;  // J/(mol K), as used with Eq. (8)
constexpr double kPi = 3.14159265358979323846;

inline int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// Flood fill over `pass` from every seed voxel, 6-connected, periodic in y and z.
void flood(int nx, int ny, int nz, const std::vector<uint8_t> &pass, const std::vector<uint8_t> &seed,
           std::vector<uint8_t> &hit) {
    const int64_t N = (int64_t)nx * ny * nz;
    hit.assign(N, 0);
    std::vector<int64_t> stack;
    stack.reserve(1024);
    for (int64_t v = 0; v < N; ++v)
        if (seed[v] && pass[v] && !hit[v]) {
            hit[v] = 1;
            stack.push_back(v);
        }
    const int64_t plane = (int64_t)nx * ny;
    while (!stack.empty()) {
        const int64_t v = stack.back();
        stack.pop_back();
        const int x = (int)(v % nx);
        const int y = (int)((v / nx) % ny);
        const int z = (int)(v / plane);
        int64_t nb[6];
        int k = 0;
        if (x > 0) nb[k++] = v - 1;
        if (x + 1 < nx) nb[k++] = v + 1;
        nb[k++] = ((int64_t)z * ny + wrap(y - 1, ny)) * nx + x;
        nb[k++] = ((int64_t)z * ny + wrap(y + 1, ny)) * nx + x;
        nb[k++] = ((int64_t)wrap(z - 1, nz) * ny + y) * nx + x;
        nb[k++] = ((int64_t)wrap(z + 1, nz) * ny + y) * nx + x;
        for (int i = 0; i < k; ++i) {
            const int64_t t = nb[i];
            if (pass[t] && !hit[t]) {
                hit[t] = 1;
                stack.push_back(t);
            }
        }
    }
}

// The device's share of prepare(): scratch layout (each part 256-byte aligned) and
// the two calls.  Every status is an LBM_* code.
size_t align256(size_t n) { return (n + 255) / 256 * 256; }

struct ScratchParts {
    size_t dp, pore, pass, hit, total;
};

ScratchParts scratch_parts(int64_t Ns, int64_t N) {
    ScratchParts s{};
    s.dp = 0;
    s.pore = align256(sizeof(double) * (size_t)Ns);
    s.pass = s.pore + align256((size_t)Ns);
    s.hit = s.pass + align256((size_t)N);
    s.total = s.hit + align256((size_t)N);
    return s;
}

int device_pore_size(const DeviceAssist &d, int nx, int ny, int nz, const std::vector<uint8_t> &pore,
                     std::vector<double> &dp, const ScratchParts &sp) {
    const int64_t N = (int64_t)nx * ny * nz;
    hipStream_t st = static_cast<hipStream_t>(d.stream);
    char *base = static_cast<char *>(d.scratch);
    hipError_t e = hipMemcpyAsync(base + sp.pore, pore.data(), (size_t)N, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return record_error(e, "device pore size: upload");
    const int s = lbm_pore_size_device(reinterpret_cast<const uint8_t *>(base + sp.pore), nx, ny, nz,
                                       reinterpret_cast<double *>(base + sp.dp), d.stream);
    if (s != LBM_OK) return s;
    dp.resize((size_t)N);
    e = hipMemcpyAsync(dp.data(), base + sp.dp, sizeof(double) * (size_t)N, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return record_error(e, "device pore size: download");
}

// hit = pass voxels connected to the x = 0 face (faces & 1) and/or x = nx - 1 (faces & 2)
int device_reach(const DeviceAssist &d, int nx, int ny, int nz, const std::vector<uint8_t> &pass, int faces,
                 std::vector<uint8_t> &hit, const ScratchParts &sp, bool upload) {
    const int64_t N = (int64_t)nx * ny * nz;
    hipStream_t st = static_cast<hipStream_t>(d.stream);
    char *base = static_cast<char *>(d.scratch);
    hipError_t e = hipSuccess;
    if (upload) e = hipMemcpyAsync(base + sp.pass, pass.data(), (size_t)N, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return record_error(e, "device reach: upload");
    const int s = lbm_reach_device(reinterpret_cast<const uint8_t *>(base + sp.pass), nx, ny, nz, faces,
                                   reinterpret_cast<uint8_t *>(base + sp.hit), nullptr, d.stream);
    if (s != LBM_OK) return s;
    hit.resize((size_t)N);
    e = hipMemcpyAsync(hit.data(), base + sp.hit, (size_t)N, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return record_error(e, "device reach: download");
}

}  // namespace

size_t prep_scratch_bytes(const lbm_grid &g, const lbm_params &p) {
    const int res = (p.mode == LBM_MODE_REACT && p.reservoir_plane) ? 1 : 0;
    const int64_t Ns = (int64_t)g.nx * g.ny * g.nz, N = (int64_t)(g.nx + res) * g.ny * g.nz;
    return scratch_parts(Ns, N).total;
}

// Pore size by 13-direction averaging (Section 2.1.3).  For each direction the
// lines are scanned once: every maximal run of pore voxels is measured from its
// first voxel and its length (voxels x |d|) credited to all its voxels.  Lines with
// no x component are closed loops under the periodic y/z wrap; a loop that is pore
// everywhere has no first voxel and is credited its full length.
void pore_size_13(int nx, int ny, int nz, const uint8_t *pore, std::vector<double> &dp) {
    static const int D[13][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1},  {1, 1, 0},  {1, -1, 0},
                                 {1, 0, 1}, {1, 0, -1}, {0, 1, 1}, {0, 1, -1}, {1, 1, 1},
                                 {1, 1, -1}, {1, -1, 1}, {-1, 1, 1}};
    const int64_t N = (int64_t)nx * ny * nz;
    dp.assign(N, 0.0);
    std::vector<uint8_t> seen(N);
    auto at = [&](int x, int y, int z) { return ((int64_t)z * ny + y) * nx + x; };
    for (int d = 0; d < 13; ++d) {
        const int dx = D[d][0], dy = D[d][1], dz = D[d][2];
        const double len = std::sqrt((double)(dx * dx + dy * dy + dz * dz));
        std::fill(seen.begin(), seen.end(), 0);
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const int64_t v = at(x, y, z);
                    if (!pore[v]) continue;
                    const int px = x - dx;
                    if (px >= 0 && px < nx && pore[at(px, wrap(y - dy, ny), wrap(z - dz, nz))]) continue;
                    // v starts a run: measure it, then credit it
                    int64_t count = 0;
                    int cx = x, cy = y, cz = z;
                    while (cx >= 0 && cx < nx && pore[at(cx, cy, cz)]) {
                        ++count;
                        cx += dx;
                        cy = wrap(cy + dy, ny);
                        cz = wrap(cz + dz, nz);
                    }
                    cx = x, cy = y, cz = z;
                    for (int64_t k = 0; k < count; ++k) {
                        const int64_t t = at(cx, cy, cz);
                        dp[t] += count * len;
                        seen[t] = 1;
                        cx += dx;
                        cy = wrap(cy + dy, ny);
                        cz = wrap(cz + dz, nz);
                    }
                }
        if (dx == 0) {
            const int64_t loop = (dy != 0 && dz != 0) ? std::lcm((int64_t)ny, (int64_t)nz) : (dy ? ny : nz);
            for (int64_t v = 0; v < N; ++v)
                if (pore[v] && !seen[v]) dp[v] += loop * len;
        }
    }
    for (int64_t v = 0; v < N; ++v) dp[v] /= 13.0;
}

int prepare(const lbm_grid &g, const uint8_t *phase, const lbm_params &p, Prepared &o, const DeviceAssist *dev) {
    if (g.nx <= 0 || g.ny <= 0 || g.nz <= 0 || !phase) return LBM_ERR_INVALID_ARG;
    if (p.struct_size != sizeof(lbm_params)) return LBM_ERR_INVALID_ARG;
    if (p.mode < LBM_MODE_DEFF || p.mode > LBM_MODE_PROTON) return LBM_ERR_INVALID_ARG;
    if (!(p.w0 > 0.0 && p.w0 < 1.0) || !(p.tau_ref > 0.5) || !(p.k_lat >= 0.0)) return LBM_ERR_INVALID_ARG;
    if (p.check_every < 2 || (p.check_every & 1) || p.max_steps < 0) return LBM_ERR_INVALID_ARG;
    if (p.knudsen && !(g.voxel_m > 0.0 && p.T_K > 0.0 && p.M_kg_mol > 0.0)) return LBM_ERR_INVALID_ARG;
    if (p.mode != LBM_MODE_PROTON && !(p.T_K > 0.0 && p.p_atm > 0.0 && p.d_ionomer_rel > 0.0))
        return LBM_ERR_INVALID_ARG;
    // the segment table packs row segment, y and z in 16 bits each
    if ((int64_t)g.nx + 1 > (int64_t)kSeg * 65535 || g.ny > 65535 || g.nz > 65535) return LBM_ERR_INVALID_ARG;
    const int64_t Ns = (int64_t)g.nx * g.ny * g.nz;
    for (int64_t v = 0; v < Ns; ++v)
        if (phase[v] > LBM_IONOMER) return LBM_ERR_BAD_PHASE;

    o = Prepared{};
    o.params = p;
    o.mode = p.mode;
    o.knudsen = p.knudsen != 0 && p.mode != LBM_MODE_PROTON;
    o.w0 = p.w0;
    o.w1 = (1.0 - p.w0) / 6.0;
    const bool react = p.mode == LBM_MODE_REACT;
    const int res = (react && p.reservoir_plane) ? 1 : 0;
    o.nx_struct = g.nx;
    o.nx = g.nx + res;
    o.ny = g.ny;
    o.nz = g.nz;
    const int nx = o.nx, ny = o.ny, nz = o.nz;
    const int64_t N = (int64_t)nx * ny * nz;
    const ScratchParts sp = scratch_parts(Ns, N);
    if (dev && (!dev->scratch || dev->bytes < sp.total || (reinterpret_cast<uintptr_t>(dev->scratch) & 255)))
        return LBM_ERR_WORKSPACE;
    std::unique_lock<std::mutex> dev_lock;  // held while this call uses the shared scratch
    auto lock_device = [&]() {
        if (dev && dev->mu && !dev_lock.owns_lock()) dev_lock = std::unique_lock<std::mutex>(*dev->mu);
    };

    // phase of the simulated grid (the reservoir plane is pore)
    std::vector<uint8_t> ph(N);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y) {
            uint8_t *dst = &ph[((int64_t)z * ny + y) * nx];
            const uint8_t *src = &phase[((int64_t)z * ny + y) * g.nx];
            if (res) dst[0] = LBM_PORE;
            std::copy(src, src + g.nx, dst + res);
        }

    o.phase = ph;

    // transport phases: pore + ionomer carry O2 (Eq. 15); ionomer alone carries protons
    std::vector<uint8_t> transport(N);
    for (int64_t v = 0; v < N; ++v)
        transport[v] = p.mode == LBM_MODE_PROTON ? ph[v] == LBM_IONOMER
                                                 : (ph[v] == LBM_PORE || ph[v] == LBM_IONOMER);

    // local diffusivity
    std::vector<double> D(N, 0.0);
    if (p.mode == LBM_MODE_PROTON) {
        o.d0 = 1.0;
        for (int64_t v = 0; v < N; ++v) D[v] = transport[v] ? 1.0 : 0.0;
    } else {
        const double Db = 0.22e-4 * std::pow(p.T_K / 293.2, 1.5) / p.p_atm;  // Eq. (7)
        o.d0 = Db;
        std::vector<double> dp;
        if (o.knudsen) {
            std::vector<uint8_t> pore(Ns);
            for (int64_t v = 0; v < Ns; ++v) pore[v] = phase[v] == LBM_PORE;
            if (dev) {
                lock_device();
                const int ds = device_pore_size(*dev, g.nx, g.ny, g.nz, pore, dp, sp);
                if (ds != LBM_OK) return ds;
            } else {
                pore_size_13(g.nx, g.ny, g.nz, pore.data(), dp);
            }
        }
        const double kn_coef = std::sqrt(8.0 * kR * p.T_K / (kPi * p.M_kg_mol)) / 3.0;  // Eq. (8)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const int64_t v = ((int64_t)z * ny + y) * nx + x;
                    if (ph[v] == LBM_IONOMER) {
                        D[v] = p.d_ionomer_rel * Db;
                    } else if (ph[v] == LBM_PORE) {
                        if (o.knudsen && x >= res) {
                            const int64_t vs = ((int64_t)z * ny + y) * g.nx + (x - res);
                            const double Dkn = kn_coef * dp[vs] * g.voxel_m;
                            D[v] = 1.0 / (1.0 / Dkn + 1.0 / Db);  // Eq. (9)
                        } else {
                            D[v] = Db;
                        }
                    }
                }
    }

    // connected to a Dirichlet face (inlet and outlet; inlet only when reacting)
    std::vector<uint8_t> seed(N, 0), left(N, 0);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y) {
            const int64_t r = ((int64_t)z * ny + y) * nx;
            seed[r] = left[r] = 1;
            if (!react) seed[r + nx - 1] = 1;
        }
    if (dev) {
        lock_device();
        const int ds = device_reach(*dev, nx, ny, nz, transport, react ? 1 : 3, o.active, sp, true);
        if (ds != LBM_OK) return ds;
    } else {
        flood(nx, ny, nz, transport, seed, o.active);
    }
    if (react) {
        o.percolates = std::any_of(o.active.begin(), o.active.end(), [](uint8_t a) { return a != 0; });
    } else {
        std::vector<uint8_t> fromleft;
        if (dev) {
            const int ds = device_reach(*dev, nx, ny, nz, transport, 1, fromleft, sp, false);
            if (ds != LBM_OK) return ds;
        } else {
            flood(nx, ny, nz, transport, left, fromleft);
        }
        o.percolates = false;
        for (int64_t r = 0; r < (int64_t)ny * nz && !o.percolates; ++r)
            if (fromleft[r * nx + nx - 1]) o.percolates = true;
    }

    if (dev_lock.owns_lock()) dev_lock.unlock();

    // D_ref and tau (Eq. 24 with tau_ref at D_ref)
    double dmax = 0.0;
    for (int64_t v = 0; v < N; ++v)
        if (o.active[v]) dmax = std::max(dmax, D[v]);
    o.d_ref = p.d_ref_rel > 0.0 ? p.d_ref_rel * o.d0 : (dmax > 0.0 ? dmax : o.d0);
    const double cs2 = (1.0 - p.w0) / 3.0;
    o.d0_lat = cs2 * (p.tau_ref - 0.5) * o.d0 / o.d_ref;
    o.omega_dense.assign(N, 0.f);
    for (int64_t v = 0; v < N; ++v)
        if (o.active[v]) {
            const double tau = 0.5 + (p.tau_ref - 0.5) * D[v] / o.d_ref;
            if (!(tau > 0.5)) return LBM_ERR_UNSTABLE;
            o.omega_dense[v] = (float)(1.0 / tau);
        }
    if (!o.knudsen) {
        const double Dp = p.mode == LBM_MODE_PROTON ? 0.0 : o.d0;
        const double Di = p.mode == LBM_MODE_PROTON ? 1.0 : p.d_ionomer_rel * o.d0;
        o.om_pore = (float)(1.0 / (0.5 + (p.tau_ref - 0.5) * Dp / o.d_ref));
        o.om_ion = (float)(1.0 / (0.5 + (p.tau_ref - 0.5) * Di / o.d_ref));
    }

    // catalyst face neighbours (Eq. 18a); periodic y, z; nothing beyond the x faces
    o.n_cat.assign(N, 0);
    auto is_cat = [&](int64_t v) { return (p.catalyst_phases >> ph[v]) & 1u; };
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int64_t v = ((int64_t)z * ny + y) * nx + x;
                int n = 0;
                if (x > 0) n += is_cat(v - 1);
                if (x + 1 < nx) n += is_cat(v + 1);
                n += is_cat(((int64_t)z * ny + wrap(y - 1, ny)) * nx + x);
                n += is_cat(((int64_t)z * ny + wrap(y + 1, ny)) * nx + x);
                n += is_cat(((int64_t)wrap(z - 1, nz) * ny + y) * nx + x);
                n += is_cat(((int64_t)wrap(z + 1, nz) * ny + y) * nx + x);
                o.n_cat[v] = (uint8_t)n;
                if (react && o.active[v] && ((p.reactive_fluids >> ph[v]) & 1u) && p.k_lat * n >= 1.0)
                    return LBM_ERR_UNSTABLE;
            }

    // segments (see Prepared), their bitmasks and compact indices
    o.nsx = (nx + kSeg - 1) / kSeg;
    o.flat = nx > kSeg && nx % kSeg == 1;
    o.win_v0.clear();
    o.win_len.clear();
    auto tile = [&](int64_t a, int64_t b) {  // windows over grid indices [a, b)
        for (int64_t v = a; v < b; v += kSeg) {
            o.win_v0.push_back((uint32_t)v);
            o.win_len.push_back((uint8_t)std::min<int64_t>(kSeg, b - v));
        }
    };
    const int64_t plane = (int64_t)ny * nx;
    if (N >= (int64_t)UINT32_MAX) return LBM_ERR_INVALID_ARG;
    for (int z = 0; z < nz; ++z) {
        const int64_t p0 = (int64_t)z * plane;
        if (!o.flat) {
            for (int64_t r = 0; r < ny; ++r) tile(p0 + r * nx, p0 + (r + 1) * nx);
        } else {
            // rows 0, 1 .. ny - 2 and ny - 1 apart (y wraps between them)
            const int64_t cut1 = std::min<int64_t>(1, ny - 1), cut2 = std::max<int64_t>(cut1, ny - 1);
            tile(p0, p0 + cut1 * nx);
            tile(p0 + cut1 * nx, p0 + cut2 * nx);
            tile(p0 + cut2 * nx, p0 + plane);
        }
    }
    o.nseg = (int64_t)o.win_v0.size();
    o.m_fluid.assign(o.nseg, 0);
    o.m_ion.assign(o.nseg, 0);
    o.m_react.assign(o.nseg, 0);
    o.m_cat.assign(o.nseg, 0);
    o.prefix.assign(o.nseg, 0);
    int64_t count = 0;
    for (int64_t sg = 0; sg < o.nseg; ++sg) {
        const int64_t base = o.win_v0[sg];
        const int len = o.win_len[sg];
        uint64_t mf = 0, mi = 0, mr = 0, mc = 0;
        for (int l = 0; l < len; ++l) {
            const int64_t v = base + l;
            const uint64_t bit = 1ull << l;
            if (o.active[v]) {
                mf |= bit;
                if (ph[v] == LBM_IONOMER) mi |= bit;
                if (react && ((p.reactive_fluids >> ph[v]) & 1u)) mr |= bit;
            }
            if (is_cat(v)) mc |= bit;
        }
        if (count > (int64_t)UINT32_MAX) return LBM_ERR_INVALID_ARG;
        o.prefix[sg] = (uint32_t)count;
        o.m_fluid[sg] = mf;
        o.m_ion[sg] = mi;
        o.m_react[sg] = mr;
        o.m_cat[sg] = mc;
        count += __builtin_popcountll(mf);
    }
    o.n_fluid = count;
    if (o.knudsen) {
        o.omega_c.resize(count);
        int64_t j = 0;
        for (int64_t v = 0; v < N; ++v)
            if (o.active[v]) o.omega_c[j++] = o.omega_dense[v];
    }
    // shift of the stored populations: the empty-box profile between the Dirichlet
    // faces (voxel centres at x + 1/2), or half the inlet value when reacting
    if (react) {
        o.sh0 = 0.5 * p.c_in;
        o.slope = 0.0;
    } else {
        o.slope = (p.c_in - p.c_out) / nx;
        o.sh0 = p.c_in - 0.5 * o.slope;
    }
    return LBM_OK;
}

void pore_depth(const Prepared &p, uint8_t *depth) {
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int64_t N = (int64_t)nx * ny * nz;
    const bool react = p.mode == LBM_MODE_REACT;
    // pores joined to a Dirichlet face through pores
    std::vector<uint8_t> pore(N), seed(N, 0), joined;
    for (int64_t v = 0; v < N; ++v) pore[v] = p.active[v] && p.phase[v] == LBM_PORE;
    for (int64_t r = 0; r < (int64_t)ny * nz; ++r) {
        seed[r * nx] = 1;
        if (!react) seed[r * nx + nx - 1] = 1;
    }
    flood(nx, ny, nz, pore, seed, joined);
    // breadth-first distance from them through the active voxels
    std::fill(depth, depth + N, (uint8_t)255);
    std::vector<int64_t> cur, next;
    for (int64_t v = 0; v < N; ++v)
        if (joined[v]) {
            depth[v] = 0;
            cur.push_back(v);
        }
    const int64_t plane = (int64_t)nx * ny;
    for (int d = 1; d <= 254 && !cur.empty(); ++d) {
        next.clear();
        for (const int64_t v : cur) {
            const int x = (int)(v % nx);
            const int y = (int)((v / nx) % ny);
            const int z = (int)(v / plane);
            int64_t nb[6];
            int k = 0;
            if (x > 0) nb[k++] = v - 1;
            if (x + 1 < nx) nb[k++] = v + 1;
            nb[k++] = ((int64_t)z * ny + wrap(y - 1, ny)) * nx + x;
            nb[k++] = ((int64_t)z * ny + wrap(y + 1, ny)) * nx + x;
            nb[k++] = ((int64_t)wrap(z - 1, nz) * ny + y) * nx + x;
            nb[k++] = ((int64_t)wrap(z + 1, nz) * ny + y) * nx + x;
            for (int i = 0; i < k; ++i) {
                const int64_t t = nb[i];
                if (p.active[t] && depth[t] == 255) {
                    depth[t] = (uint8_t)d;
                    next.push_back(t);
                }
            }
        }
        cur.swap(next);
    }
}

}  // namespace cl
