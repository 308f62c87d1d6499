// Solver engine behind the C ABI of include/lbm.h: workspace layout, block
// tables, HIP-graph-captured check windows, per-instance convergence control.
//
// A single solver is an engine with one instance; the batched form is the same
// engine with many instances concatenated (segments, compact fluid arrays) and
// one launch per step covering every live instance.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <thread>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <memory>
#include <new>
#include <vector>

#include "kernels.h"
#include "prep.h"

namespace cl {
namespace {

constexpr size_t kAlign = 256;
constexpr int kMeasMaxBlocks = 512;
constexpr int kMeasWaves = 4;
constexpr int64_t kMaxWindow = int64_t(1) << 22;  // longest check window (steps)

size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

thread_local char g_last_error[256] = "";

// record the first failing HIP call of an operation (read by lbm_last_error)
hipError_t note(hipError_t e, const char *what) {
    if (e != hipSuccess) snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%d)", what, hipGetErrorName(e), (int)e);
    return e;
}

struct RunState {
    lbm_run_info info{};
    double q_prev = 0, m_prev = 0;  // output and mass at the previous check
    double dm_prev = 0;             // mass change over the previous window
    int64_t k_prev = 0;             // length of the previous window (0: none)
    int have_prev = 0;
    int slow = 0;                   // mass decays by less than half per window
    int done = 0;
    int measured = 0;
};

struct Engine {
    std::vector<Prepared> P;
    int mode = 0;
    bool knudsen = false, react = false;
    int ninst = 0;
    int64_t nseg_total = 0, nf_total = 0, stride = 0;
    std::vector<int64_t> seg_base, fluid_base, dense_base;
    int check_every = 1000;

    // workspace
    size_t ws_need = 0;
    size_t off_zbase = 0;  // per-instance zeros: dense output on one instance's own grid
    std::vector<int> cb_start, cb_count;  // conversion blocks of each instance
    size_t off_f0 = 0, off_f1 = 0, off_om = 0, off_snap = 0, off_rec = 0, off_inst = 0, off_dbase = 0, off_sblk = 0,
           off_sinst = 0,
           off_cblk = 0, off_mblk = 0, off_rng = 0, off_part = 0, off_res = 0;
    int64_t cap_sblk = 0, cap_cblk = 0, cap_mblk = 0;

    bool bound = false;
    int device = 0;
    hipStream_t st = nullptr;
    char *ws = nullptr;
    double *res_host = nullptr;
    Lattice L{};
    float *f[2] = {nullptr, nullptr};
    float *csnap = nullptr;
    int cur = 0;

    static constexpr int kXcds = 8;  // MI355X: 8 XCDs, each with its own L2
    int waves = 4, spw = 1, xcd = 1;
    // Rows per y slab of the one-instance step list (0: grid order); set at creation.
    int slab_rows = 0;
    // Alternate the direction in which one-step launches walk the segment list.
    int alt_order = 1;
    // Two steps per launch (one instance only): rows per tile (0 = off), planes per chunk.
    int t2_by = 0, t2_zc = 32;
    // Batches run as consecutive groups of instances whose combined working set
    // (both lattices, 1/tau, snapshot, records) fits this many bytes, so each group
    // stays in the 256 MB last-level cache (Infinity Cache) while it steps; 0 runs
    // every instance together.
    int64_t group_bytes = int64_t(192) << 20;
    int step_nblk = 0, step_nent = 0, meas_nblk = 0, conv_nblk = 0;
    std::vector<int> live;
    std::vector<RunState> rs;

    // Captured check windows, one per starting lattice: a window whose launch count
    // is odd ends on the other lattice, so its next replay needs the other graph.
    // g_valid is cleared whenever the launch form or tables change; both slots are
    // re-captured lazily after that.
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int g_nblk[2] = {-1, -1}, g_k[2] = {-1, -1};
    bool g_slot[2] = {false, false};
    bool g_valid = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;  // bracket the step launches of a window
    bool ev_pending = false;
    int64_t ev_launches = 0;

    ~Engine() {
        drop_graphs();
        if (res_host) (void)hipHostFree(res_host);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
    }

    template <typename T>
    T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }

    void layout() {
        nseg_total = nf_total = 0;
        seg_base.resize(ninst);
        fluid_base.resize(ninst);
        dense_base.resize(ninst);
        int64_t dense = 0;
        for (int i = 0; i < ninst; ++i) {
            seg_base[i] = nseg_total;
            fluid_base[i] = nf_total;
            dense_base[i] = dense;
            nseg_total += P[i].nseg;
            nf_total += P[i].n_fluid;
            dense += (int64_t)P[i].nx * P[i].ny * P[i].nz;
        }
        stride = (int64_t)align_up((size_t)std::max<int64_t>(nf_total, 1), 64);
        cap_sblk = nseg_total;
        cap_cblk = nseg_total / 4 + ninst + 1;
        cap_mblk = (int64_t)ninst * kMeasMaxBlocks;
        size_t o = 0;
        auto take = [&](size_t bytes) {
            const size_t r = o;
            o = align_up(o + std::max<size_t>(bytes, 1));
            return r;
        };
        off_f0 = take(sizeof(float) * 7 * stride);
        off_f1 = take(sizeof(float) * 7 * stride);
        off_om = knudsen ? take(sizeof(float) * stride) : 0;
        off_snap = take(sizeof(float) * stride);
        off_rec = take(sizeof(SegRec) * nseg_total);
        off_inst = take(sizeof(InstDev) * ninst);
        off_dbase = take(sizeof(int64_t) * ninst);
        off_zbase = take(sizeof(int64_t) * ninst);
        off_sblk = take(sizeof(uint32_t) * cap_sblk);
        off_sinst = take(sizeof(uint32_t) * (ninst > 1 ? cap_sblk : 1));
        off_cblk = take(sizeof(int2) * cap_cblk);
        off_mblk = take(sizeof(int4) * cap_mblk);
        off_rng = take(sizeof(int2) * ninst);
        off_part = take(sizeof(double) * NQ * cap_mblk);
        off_res = take(sizeof(double) * NQ * ninst);
        ws_need = o;
    }

    InstDev inst_dev(int i) const {
        const Prepared &p = P[i];
        InstDev d{};
        d.nx = p.nx;
        d.ny = p.ny;
        d.nz = p.nz;
        d.nsx = p.nsx;
        d.seg_base = seg_base[i];
        d.nseg = p.nseg;
        d.sh0 = p.sh0;
        d.slope = p.slope;
        d.w0 = p.w0;
        d.w1 = p.w1;
        d.pull_dx = p.w1 * p.slope;
        d.abb_in = 2.0 * p.w1 * (p.params.c_in - p.sh0);
        d.abb_out = 2.0 * p.w1 * (p.params.c_out - (p.sh0 - p.slope * (p.nx - 1)));
        d.k = p.params.k_lat;
        d.om_pore = p.om_pore;
        d.om_ion = p.om_ion;
        return d;
    }

    hipError_t upload_tables() {
        // step list: the segments holding fluid of every live instance, in grid order
        std::vector<uint32_t> sb, si;
        for (int i : live) {
            const Prepared &p = P[i];
            for (int64_t g = 0; g < p.nseg; ++g)
                if (p.m_fluid[g]) {
                    sb.push_back((uint32_t)(seg_base[i] + g));
                    if (ninst > 1) si.push_back((uint32_t)i);
                }
        }
        // One instance: walk it as kXcds slabs of consecutive rows in y, each slab
        // plane by plane in z.  With the XCD-aware block order each XCD then steps
        // one slab, and the rows a segment pulls from (y -+ 1 in its plane, the
        // same row in z -+ 1) were touched a slab plane earlier, a few hundred
        // segments back, still in that XCD's L2.  In grid order an XCD steps a slab
        // of whole planes, and the plane before is too far back for its L2.
        if (live.size() == 1 && slab_rows > 0) {
            const Prepared &p = P[live[0]];
            const int64_t nx = p.nx, ny = p.ny, nz = p.nz, plane = ny * nx;
            const int64_t base = seg_base[live[0]], yb = slab_rows;
            auto key = [&](uint32_t gs) {  // (slab of the window's first row, plane, grid index)
                const int64_t v0 = p.win_v0[(int64_t)gs - base];
                const int64_t row = v0 / nx, y = row % ny, z = row / ny;
                return ((y / yb) * nz + z) * plane + (v0 - z * plane);
            };
            std::sort(sb.begin(), sb.end(), [&](uint32_t a, uint32_t b) { return key(a) < key(b); });
        }
        step_nent = (int)sb.size();
        const int per = waves * spw;
        step_nblk = (step_nent + per - 1) / per;
        // measure table and per-instance partial ranges
        std::vector<int4> mb;
        std::vector<int2> rg(ninst, make_int2(0, 0));
        for (int i : live) {
            int64_t nb = (P[i].nseg + kMeasWaves * 16 - 1) / (kMeasWaves * 16);
            nb = std::max<int64_t>(1, std::min<int64_t>(nb, kMeasMaxBlocks));
            rg[i] = make_int2((int)mb.size(), (int)nb);
            for (int64_t b = 0; b < nb; ++b) mb.push_back(make_int4(i, (int)b, (int)nb, (int)mb.size()));
        }
        meas_nblk = (int)mb.size();
        hipError_t e = hipSuccess;
        if (!sb.empty())
            e = hipMemcpyAsync(at<uint32_t>(off_sblk), sb.data(), sizeof(uint32_t) * sb.size(), hipMemcpyHostToDevice, st);
        if (e == hipSuccess && !si.empty())
            e = hipMemcpyAsync(at<uint32_t>(off_sinst), si.data(), sizeof(uint32_t) * si.size(), hipMemcpyHostToDevice,
                               st);
        if (e == hipSuccess && !mb.empty())
            e = hipMemcpyAsync(at<int4>(off_mblk), mb.data(), sizeof(int4) * mb.size(), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(at<int2>(off_rng), rg.data(), sizeof(int2) * ninst, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);  // host vectors go out of scope
        g_valid = false;
        return e;
    }

    // Segment records of instance i (see SegRec and Prepared): masks and compact
    // prefixes of the window and of its four neighbour windows (the same lanes
    // moved one row in y or one plane in z, periodic), and the reaction bit planes.
    void build_records(int i, SegRec *out) const {
        const Prepared &p = P[i];
        const int nx = p.nx, ny = p.ny, nz = p.nz;
        const int64_t N = (int64_t)nx * ny * nz, plane = (int64_t)ny * nx;
        // the fluid map as a bit string in grid order, and its rank per word
        const int64_t nw = N / 64 + 2;
        std::vector<uint64_t> fb(nw, 0ull);
        std::vector<int64_t> rank(nw, 0);
        for (int64_t v = 0; v < N; ++v)
            if (p.active[v]) fb[v >> 6] |= 1ull << (v & 63);
        for (int64_t w = 1; w < nw; ++w) rank[w] = rank[w - 1] + __builtin_popcountll(fb[w - 1]);
        auto bits = [&](int64_t pos, int len) {  // fluid bits of grid indices pos .. pos + len - 1
            const int64_t w = pos >> 6;
            const int sh = (int)(pos & 63);
            uint64_t v = fb[w] >> sh;
            if (sh) v |= fb[w + 1] << (64 - sh);
            return len >= 64 ? v : v & ((1ull << len) - 1ull);
        };
        auto rank_at = [&](int64_t pos) {  // fluid voxels before grid index pos
            const int sh = (int)(pos & 63);
            return rank[pos >> 6] + (sh ? __builtin_popcountll(fb[pos >> 6] & ((1ull << sh) - 1ull)) : 0);
        };
        for (int64_t g = 0; g < p.nseg; ++g) {
            SegRec r{};
            const int64_t v0 = p.win_v0[g];
            const int len = p.win_len[g];
            const int64_t row = v0 / nx;
            const int x0 = (int)(v0 - row * nx), y = (int)(row % ny), z = (int)(row / ny);
            const int brk = x0 + len > nx ? nx - x0 : 64;  // first lane of the next row
            const uint64_t m = p.m_fluid[g];
            const uint64_t inside = len >= 64 ? ~0ull : (1ull << len) - 1ull;
            // lanes at x = 0 and at x = nx - 1
            uint64_t at0 = 0ull, at1 = 0ull;
            if (x0 == 0) at0 |= 1ull;
            if (brk < len) at0 |= 1ull << brk;
            if (nx - 1 - x0 < len) at1 |= 1ull << (nx - 1 - x0);
            const uint64_t before = (m << 1) | (v0 > 0 ? (fb[(v0 - 1) >> 6] >> ((v0 - 1) & 63)) & 1ull : 0ull);
            const uint64_t after = (m >> 1) | (v0 + len < N ? ((fb[(v0 + len) >> 6] >> ((v0 + len) & 63)) & 1ull) << (len - 1) : 0ull);
            r.m = m;
            r.left = before & inside & ~at0;
            r.right = after & inside & ~at1;
            const int64_t off[4] = {y == 0 ? (int64_t)(ny - 1) * nx : -(int64_t)nx,
                                    y == ny - 1 ? -(int64_t)(ny - 1) * nx : (int64_t)nx,
                                    z == 0 ? (int64_t)(nz - 1) * plane : -plane,
                                    z == nz - 1 ? -(int64_t)(nz - 1) * plane : plane};
            for (int k = 0; k < 4; ++k) {
                r.nb[k] = bits(v0 + off[k], len);
                r.pnb[k] = (uint32_t)(fluid_base[i] + rank_at(v0 + off[k]));
            }
            r.ion = p.m_ion[g];
            const uint64_t mr = p.m_react[g];
            for (int l = 0; l < len; ++l) {
                if (!((mr >> l) & 1ull)) continue;
                const int n = p.n_cat[v0 + l];
                if (n & 1) r.n0 |= 1ull << l;
                if (n & 2) r.n1 |= 1ull << l;
                if (n & 4) r.n2 |= 1ull << l;
            }
            r.pre = (uint32_t)(fluid_base[i] + p.prefix[g]);
            r.v0 = (uint32_t)v0;
            r.x0 = (uint16_t)x0;
            r.brk = (uint8_t)brk;
            r.len = (uint8_t)len;
            r.inst = (uint16_t)i;
            out[g] = r;
        }
    }

    void drop_graphs() {
        for (int c = 0; c < 2; ++c) {
            if (gexec[c]) (void)hipGraphExecDestroy(gexec[c]);
            gexec[c] = nullptr;
            g_slot[c] = false;
        }
    }

    hipError_t bind(void *mem, size_t bytes, hipStream_t stream) {
        drop_graphs();
        g_valid = false;
        ws = static_cast<char *>(mem);
        st = stream;
        g_last_error[0] = 0;
        hipError_t e = note(hipGetDevice(&device), "hipGetDevice");
        if (e != hipSuccess) return e;
        if (!res_host) {
            e = note(hipHostMalloc((void **)&res_host, sizeof(double) * NQ * ninst, hipHostMallocDefault), "hipHostMalloc");
            if (e != hipSuccess) return e;
        }
        if (!ev0 && (e = note(hipEventCreate(&ev0), "hipEventCreate")) != hipSuccess) return e;
        if (!ev1 && (e = note(hipEventCreate(&ev1), "hipEventCreate")) != hipSuccess) return e;
        f[0] = at<float>(off_f0);
        f[1] = at<float>(off_f1);
        csnap = at<float>(off_snap);
        L.rec = at<SegRec>(off_rec);
        L.omega = knudsen ? at<float>(off_om) : nullptr;
        L.inst = at<InstDev>(off_inst);
        L.stride = (uint32_t)stride;
        // metadata (host staging, then one synchronisation)
        cb_start.clear();
        cb_count.clear();
        std::vector<SegRec> rec(nseg_total);
        std::vector<float> om(knudsen ? nf_total : 0);
        std::vector<InstDev> id(ninst);
        std::vector<int2> cb;
        for (int i = 0; i < ninst; ++i) {
            build_records(i, rec.data() + seg_base[i]);
            const Prepared &p = P[i];
            if (knudsen) std::copy(p.omega_c.begin(), p.omega_c.end(), om.begin() + fluid_base[i]);
            id[i] = inst_dev(i);
            cb_start.push_back((int)cb.size());
            for (int64_t b = 0; b < (p.nseg + 3) / 4; ++b) cb.push_back(make_int2(i, (int)(b * 4)));
            cb_count.push_back((int)cb.size() - cb_start.back());
        }
        conv_nblk = (int)cb.size();
        const std::vector<int64_t> zeros(ninst, 0);
        auto up = [&](size_t off, const void *src, size_t n) {
            return note(n ? hipMemcpyAsync(ws + off, src, n, hipMemcpyHostToDevice, st) : hipSuccess, "upload");
        };
        if ((e = up(off_rec, rec.data(), sizeof(SegRec) * rec.size())) != hipSuccess) return e;
        if (knudsen && (e = up(off_om, om.data(), 4 * om.size())) != hipSuccess) return e;
        if ((e = up(off_inst, id.data(), sizeof(InstDev) * id.size())) != hipSuccess) return e;
        if ((e = up(off_dbase, dense_base.data(), 8 * dense_base.size())) != hipSuccess) return e;
        if ((e = up(off_zbase, zeros.data(), 8 * zeros.size())) != hipSuccess) return e;
        if ((e = up(off_cblk, cb.data(), sizeof(int2) * cb.size())) != hipSuccess) return e;
        if ((e = note(hipStreamSynchronize(st), "bind sync")) != hipSuccess) return e;
        bound = true;
        live.clear();
        for (int i = 0; i < ninst; ++i) live.push_back(i);
        if ((e = note(upload_tables(), "upload_tables")) != hipSuccess) return e;
        return note(init(nullptr), "init");
    }

    hipError_t init(const float *c_dense) {
        cur = 0;
        rs.assign(ninst, RunState{});
        for (auto &r : rs) r.info.status = LBM_NOT_CONVERGED;
        live.clear();
        for (int i = 0; i < ninst; ++i) live.push_back(i);
        hipError_t e = upload_tables();
        if (e != hipSuccess) return e;
        return note(launch_init_eq(L, conv_nblk, at<int2>(off_cblk), react, c_dense, at<int64_t>(off_dbase), f[0], csnap, st),
                    "k_init_eq launch");
    }

    // the user-level step/measure calls act on every instance
    hipError_t all_live() {
        if ((int)live.size() == ninst) return hipSuccess;
        live.clear();
        for (int i = 0; i < ninst; ++i) live.push_back(i);
        return upload_tables();
    }

    StepLaunch step_launch() const {
        StepLaunch s{};
        s.waves = waves;
        s.spw = spw;
        s.xcd = xcd;
        s.nblk = step_nblk;
        s.nent = step_nent;
        s.list = at<uint32_t>(off_sblk);
        s.list_inst = at<uint32_t>(off_sinst);
        s.single = ninst == 1 ? 1 : 0;
        return s;
    }

    bool two_step() const { return t2_by > 0 && ninst == 1; }
    // the two-step kernel tiles rows of segments: the row layout only (Prepared)
    bool two_step_possible() const { return ninst == 1 && !P[0].flat; }

    Step2Launch step2_launch() const {
        const Prepared &p = P[0];
        Step2Launch s{};
        s.by = t2_by;
        s.zc = t2_zc;
        s.nty = (p.ny + t2_by - 1) / t2_by;
        s.ncz = (p.nz + t2_zc - 1) / t2_zc;
        s.nblk = p.nsx * s.nty * s.ncz;
        s.xcd = xcd;
        return s;
    }

    // Lattice swaps made by n steps, mod 2: one per launch.
    int flips(int64_t n) const { return (int)((two_step() ? n / 2 + (n & 1) : n) & 1); }

    hipError_t steps(int64_t n) {
        int64_t k = 0;
        if (two_step()) {
            const Step2Launch s2 = step2_launch();
            for (; k + 2 <= n; k += 2) {
                hipError_t e = launch_step2(L, s2, knudsen, react, f[cur], f[cur ^ 1], st);
                if (e != hipSuccess) return e;
                cur ^= 1;
            }
        }
        StepLaunch s = step_launch();
        for (; k < n; ++k) {
            s.reverse = alt_order ? (int)(k & 1) : 0;
            hipError_t e = launch_step(L, s, knudsen, react, f[cur], f[cur ^ 1], st);
            if (e != hipSuccess) return e;
            cur ^= 1;
        }
        return hipSuccess;
    }

    hipError_t measure_enqueue(int update_snap) {
        MeasureLaunch m{};
        m.nblk = meas_nblk;
        m.blk = at<int4>(off_mblk);
        m.partial = at<double>(off_part);
        m.update_snap = update_snap;
        m.csnap = csnap;
        hipError_t e = launch_measure(L, m, react, f[cur], st);
        if (e != hipSuccess) return e;
        return launch_finish(at<double>(off_part), at<int2>(off_rng), ninst, at<double>(off_res), st);
    }

    hipError_t read_results() {
        hipError_t e = hipMemcpyAsync(res_host, at<double>(off_res), sizeof(double) * NQ * ninst, hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(st);
    }

    // Capture K0 steps starting from lattice `from` into graph slot `from`.
    hipError_t capture(int K0, int from) {
        if (gexec[from]) {
            (void)hipGraphExecDestroy(gexec[from]);
            gexec[from] = nullptr;
        }
        g_slot[from] = false;
        hipGraph_t graph = nullptr;
        hipError_t e = note(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        if (e != hipSuccess) return e;
        const int c0 = cur;
        cur = from;
        hipError_t e1 = steps(K0);
        cur = c0;
        e = note(hipStreamEndCapture(st, &graph), "hipStreamEndCapture");
        if (e1 != hipSuccess) return e1;
        if (e != hipSuccess) return e;
        e = note(hipGraphInstantiate(&gexec[from], graph, nullptr, nullptr, 0), "hipGraphInstantiate");
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return e;
        g_slot[from] = true;
        g_nblk[from] = step_nblk;
        g_k[from] = K0;
        return hipSuccess;
    }

    // One check window: `reps` replays of a captured graph of K0 steps, then the
    // FP64 reductions (which also refresh the concentration snapshot).  When K0
    // steps take an odd number of launches (the two-step form with K0/2 odd), each
    // replay ends on the other lattice, so replays alternate between the graphs
    // captured from either lattice.
    hipError_t window(int K0, int64_t reps) {
        if (st == nullptr) {  // the legacy default stream cannot be captured
            for (int64_t r = 0; r < reps; ++r) {
                hipError_t e = steps(K0);
                if (e != hipSuccess) return e;
            }
            return measure_enqueue(1);
        }
        if (!g_valid) {
            drop_graphs();
            g_valid = true;
        }
        const bool fl = flips(K0) != 0;
        for (int k = 0; k < ((fl && reps > 1) ? 2 : 1); ++k) {
            const int from = cur ^ k;
            if (!g_slot[from] || g_nblk[from] != step_nblk || g_k[from] != K0) {
                hipError_t e = capture(K0, from);
                if (e != hipSuccess) return e;
            }
        }
        hipError_t e = note(hipEventRecord(ev0, st), "hipEventRecord");
        for (int64_t r = 0; r < reps && e == hipSuccess; ++r) {
            e = note(hipGraphLaunch(gexec[cur], st), "hipGraphLaunch");
            if (fl) cur ^= 1;
        }
        if (e == hipSuccess) e = note(hipEventRecord(ev1, st), "hipEventRecord");
        if (e != hipSuccess) return e;
        ev_pending = true;
        ev_launches = (int64_t)K0 * reps;
        return measure_enqueue(1);
    }

    void fill_info(int i, const double *r, int64_t K, lbm_run_info &info) const {
        const Prepared &p = P[i];
        const double A = (double)p.ny * p.nz;
        info.j_in = r[Q_JIN] / A;
        info.j_out = r[Q_JOUT] / A;
        info.j_vol = p.nx > 1 ? r[Q_JINT] / ((double)(p.nx - 1) * A) : info.j_in;
        info.rate = r[Q_RATE] / A;
        info.mass = r[Q_MASS];
        if (K > 0) info.residual = r[Q_CMAX] > 0 ? r[Q_DCMAX] / ((double)K * r[Q_CMAX]) : 0.0;
    }

    // Stop rule for one instance after a check window of K steps; true when finished.
    //
    // The iteration converges geometrically; its rate per window, rho, is taken from
    // the total mass (an FP64 sum over every voxel, far less noisy than any flux),
    // using two consecutive windows of equal length.  The remaining error of a
    // quantity that changed by d over the last window is d rho / (1 - rho).  Both the
    // output (volume-averaged flux, or total reaction rate) and the mass must be
    // within tol_flux by that estimate, and the output's last change itself too;
    // the windowed residual and the flux balance are checked as well.
    bool evaluate(int i, const double *r, int64_t K) {
        RunState &s = rs[i];
        const lbm_params &pp = P[i].params;
        lbm_run_info &info = s.info;
        fill_info(i, r, K, info);
        s.measured = 1;
        info.checks += 1;
        info.steps += K;
        if (r[Q_BAD] > 0.0) {
            info.status = LBM_ERR_DIVERGED;
            return true;
        }
        const double Q = react ? info.rate : info.j_vol;
        const double M = info.mass;
        const double inf = std::numeric_limits<double>::infinity();
        double est = inf;
        s.slow = 0;  // no rate estimate yet (or the window length just changed): keep it
        if (s.have_prev) {
            const double dq = Q - s.q_prev, dm = M - s.m_prev;
            const double rq = std::fabs(dq) / std::max(std::fabs(Q), 1e-300);
            const double rm = std::fabs(dm) / std::max(std::fabs(M), 1e-300);
            if (s.k_prev == K && s.dm_prev != 0.0) {
                const double rho = dm / s.dm_prev;
                if (rho <= 0.0 || dm == 0.0) {  // the mass change is at its noise floor
                    est = std::max(rq, rm);
                    s.slow = 0;
                } else if (rho < 1.0) {
                    const double amp = rho / (1.0 - rho);
                    est = std::max(std::max(rq, rm) * amp, rq);
                    s.slow = rho > 0.5;
                } else {
                    s.slow = 1;  // not contracting yet at this window length
                }
            } else if (dm == 0.0 && s.k_prev == K) {
                est = rq;
                s.slow = 0;
            }
            s.dm_prev = dm;
        }
        s.q_prev = Q;
        s.m_prev = M;
        s.k_prev = K;
        s.have_prev = 1;
        info.est_error = est;
        const double jref = std::max(std::fabs(info.j_in), 1e-300);
        double bal = react ? std::fabs(info.j_in - info.rate) / jref : std::fabs(info.j_in - info.j_out) / jref;
        if (std::fabs(info.j_in) < 1e-30 && std::fabs(info.j_out) < 1e-30 && std::fabs(info.rate) < 1e-30) bal = 0.0;
        const bool conv = info.checks >= 3 && est < pp.tol_flux && info.residual < pp.tol_change && bal < pp.tol_balance;
        if (conv) {
            info.status = LBM_OK;
            return true;
        }
        info.status = LBM_NOT_CONVERGED;
        return info.steps >= pp.max_steps;
    }

    // The steady-state loop.  budget caps the number of new steps (windows are
    // shortened to fit); instances still running when it is spent report
    // LBM_NOT_CONVERGED and can be resumed by another call.
    int run(lbm_run_info *out, int64_t budget = std::numeric_limits<int64_t>::max()) {
        if (!bound) return LBM_ERR_UNBOUND;
        const int K = check_every;
        int64_t spent = 0;
        // instances without a percolating path are finished before the first step
        std::vector<int> still;
        for (int i : live) {
            if (rs[i].done) continue;
            if (!react && !P[i].percolates) {
                rs[i].done = 1;
                rs[i].info.status = LBM_ERR_NO_PERCOLATION;
            } else {
                still.push_back(i);
            }
        }
        if (still.size() != live.size()) {
            live = still;
            if (upload_tables() != hipSuccess) return LBM_ERR_HIP;
        }
        int64_t reps = 1;  // window = reps * K steps; doubled while a live instance is slow
        while (!live.empty()) {
            const int64_t room = (budget - spent) / K;
            if (room < 1) break;
            reps = std::min(reps, room);
            if (window(K, reps) != hipSuccess) return LBM_ERR_HIP;
            spent += (int64_t)K * reps;
            if (read_results() != hipSuccess) return LBM_ERR_HIP;
            float win_ms = 0.f;
            if (ev_pending && hipEventElapsedTime(&win_ms, ev0, ev1) == hipSuccess) {
                for (int i : live) {
                    rs[i].info.kernel_ms += win_ms;
                    rs[i].info.kernel_launches += ev_launches;
                }
            }
            ev_pending = false;
            std::vector<int> keep;
            bool any_slow = false;
            for (int i : live) {
                if (evaluate(i, res_host + (size_t)i * NQ, (int64_t)K * reps)) {
                    rs[i].done = 1;
                } else {
                    keep.push_back(i);
                    any_slow = any_slow || rs[i].slow;
                }
            }
            if (keep.size() != live.size()) {
                live = keep;
                if (upload_tables() != hipSuccess) return LBM_ERR_HIP;
            }
            // longer windows while a live instance converges slowly (its rate estimate
            // needs windows comparable to its decay time; in a batch, instances that
            // are fast or at their rounding floor must not hold it back), but never
            // longer than 1/32 of the steps taken so far, so a stop found at the end
            // of a window overshoots the first passing check by at most about 3%
            int64_t taken = std::numeric_limits<int64_t>::max();
            for (int i : live) taken = std::min(taken, rs[i].info.steps);
            if (!live.empty() && any_slow && (int64_t)K * reps * 2 <= kMaxWindow && (int64_t)K * reps * 64 <= taken)
                reps *= 2;
        }
        int worst = LBM_OK;
        for (int i = 0; i < ninst; ++i) {
            if (out) out[i] = rs[i].info;
            const int s = rs[i].info.status;
            if (s < 0 && (worst >= 0 || s < worst)) worst = s;
            if (s == LBM_NOT_CONVERGED && worst == LBM_OK) worst = LBM_NOT_CONVERGED;
        }
        return worst;
    }

    int64_t working_bytes(int i) const {
        const Prepared &p = P[i];
        return p.n_fluid * (int64_t)(56 + 4 + (knudsen ? 4 : 0)) + p.nseg * (int64_t)(sizeof(SegRec) + 4);
    }

    // The steady-state loop over groups of pending instances (see group_bytes): each
    // group runs until all its instances finish (or the step budget is spent) before
    // the next group starts.  One instance, or group_bytes == 0: plain run().
    int run_grouped(lbm_run_info *out, int64_t budget = std::numeric_limits<int64_t>::max()) {
        if (!bound) return LBM_ERR_UNBOUND;
        if (ninst == 1 || group_bytes <= 0) return run(out, budget);
        std::vector<int> pending;
        for (int i = 0; i < ninst; ++i)
            if (!rs[i].done) pending.push_back(i);
        int64_t left = budget;
        size_t k = 0;
        while (k < pending.size() && left > 0) {
            std::vector<int> grp;
            int64_t bytes = 0;
            while (k < pending.size() && (grp.empty() || bytes + working_bytes(pending[k]) <= group_bytes)) {
                bytes += working_bytes(pending[k]);
                grp.push_back(pending[k++]);
            }
            live = grp;
            if (upload_tables() != hipSuccess) return LBM_ERR_HIP;
            int64_t s0 = 0, s1 = 0;
            for (int i : grp) s0 = std::max(s0, rs[i].info.steps);
            const int st = run(nullptr, left);
            if (st == LBM_ERR_HIP || st == LBM_ERR_UNBOUND) return st;
            bool unfinished = false;
            for (int i : grp) {
                s1 = std::max(s1, rs[i].info.steps);
                unfinished = unfinished || !rs[i].done;
            }
            left -= std::max<int64_t>(s1 - s0, 0);
            if (unfinished) break;  // the budget ran out inside this group
        }
        int worst = LBM_OK;
        for (int i = 0; i < ninst; ++i) {
            if (out) out[i] = rs[i].info;
            const int s = rs[i].info.status;
            if (s < 0 && (worst >= 0 || s < worst)) worst = s;
            if (s == LBM_NOT_CONVERGED && worst == LBM_OK) worst = LBM_NOT_CONVERGED;
        }
        return worst;
    }

    int deff(int i, double *out) const {
        const Prepared &p = P[i];
        if (react) return LBM_ERR_WRONG_MODE;
        if (!p.percolates) {
            *out = 0.0;
            return LBM_ERR_NO_PERCOLATION;
        }
        if (!rs[i].measured) return LBM_ERR_UNBOUND;
        const double dc = p.params.c_in - p.params.c_out;
        if (dc == 0.0) return LBM_ERR_INVALID_ARG;
        *out = rs[i].info.j_vol * p.nx / (dc * p.d0_lat);
        return rs[i].info.status == LBM_NOT_CONVERGED ? LBM_NOT_CONVERGED : LBM_OK;
    }

    int rate(int i, double *r, double *jin) const {
        if (!react) return LBM_ERR_WRONG_MODE;
        if (!rs[i].measured) return LBM_ERR_UNBOUND;
        if (r) *r = rs[i].info.rate;
        if (jin) *jin = rs[i].info.j_in;
        return rs[i].info.status == LBM_NOT_CONVERGED ? LBM_NOT_CONVERGED : LBM_OK;
    }

    void info_of(int i, lbm_info &o) const {
        const Prepared &p = P[i];
        o.nx = p.nx;
        o.ny = p.ny;
        o.nz = p.nz;
        o.nx_struct = p.nx_struct;
        o.n_active = p.n_fluid;
        o.n_segments = p.nseg;
        o.n_listed = 0;
        for (int64_t g = 0; g < p.nseg; ++g) o.n_listed += p.m_fluid[g] != 0ull;
        o.d0 = p.d0;
        o.d_ref = p.d_ref;
        o.d0_lat = p.d0_lat;
        o.percolates = p.percolates ? 1 : 0;
        o.mode = p.mode;
    }
};

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int now = -1;
        if (prev >= 0 && hipGetDevice(&now) == hipSuccess && now != prev) (void)hipSetDevice(prev);
    }
};

int hip_status_at(hipError_t e, const char *where) {
    if (e == hipSuccess) return LBM_OK;
    if (!g_last_error[0]) snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%d)", where, hipGetErrorName(e), (int)e);
    return LBM_ERR_HIP;
}
#define hip_status(e) hip_status_at((e), __func__)

int make_engine(int n, const lbm_grid *grids, const uint8_t *const *phases, const lbm_params *params,
                std::unique_ptr<Engine> &out, const DeviceAssist *dev = nullptr) {
    if (n <= 0 || n > 65535 || !grids || !phases || !params) return LBM_ERR_INVALID_ARG;
    auto E = std::make_unique<Engine>();
    E->ninst = n;
    E->P.resize(n);
    for (int i = 0; i < n; ++i)
        if (!phases[i]) return LBM_ERR_INVALID_ARG;
    // instances are independent: preprocess them on parallel host threads
    std::vector<int> st(n, LBM_OK);
    const int nth = std::max(1, std::min<int>(n, (int)std::thread::hardware_concurrency()));
    std::atomic<int> next{0};
    auto work = [&]() {
        for (int i = next++; i < n; i = next++) st[i] = prepare(grids[i], phases[i], params[i], E->P[i], dev);
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < nth; ++t) pool.emplace_back(work);
    work();
    for (auto &t : pool) t.join();
    for (int i = 0; i < n; ++i) {
        if (st[i] != LBM_OK) return st[i];
        if (i > 0 && (params[i].mode != params[0].mode || E->P[i].knudsen != E->P[0].knudsen))
            return LBM_ERR_INVALID_ARG;
    }
    E->mode = params[0].mode;
    E->knudsen = E->P[0].knudsen;
    E->react = E->mode == LBM_MODE_REACT;
    E->check_every = params[0].check_every;
    // one y slab of the step list per XCD, when the slabs are at least two rows
    if (n == 1 && E->P[0].ny >= 2 * Engine::kXcds)
        E->slab_rows = (E->P[0].ny + Engine::kXcds - 1) / Engine::kXcds;
    E->layout();
    // segment indices are 32-bit; population byte offsets are 32-bit (buffer resources)
    if (E->nseg_total > (int64_t)INT32_MAX || 28 * E->stride >= ((int64_t)1 << 32) - 64) return LBM_ERR_INVALID_ARG;
    E->rs.assign(n, RunState{});
    out = std::move(E);
    return LBM_OK;
}

}  // namespace

int record_error(hipError_t e, const char *where) { return hip_status_at(e, where); }

}  // namespace cl

struct lbm_solver {
    std::unique_ptr<cl::Engine> E;
};
struct lbm_batch {
    std::unique_ptr<cl::Engine> E;
};

#define LBM_GUARD_BEGIN try {
#define LBM_GUARD_END                     \
    }                                     \
    catch (const std::bad_alloc &) {      \
        return LBM_ERR_INVALID_ARG;       \
    }                                     \
    catch (...) {                         \
        return LBM_ERR_INVALID_ARG;       \
    }

extern "C" {

int lbm_params_default(lbm_params *p) {
    if (!p) return LBM_ERR_INVALID_ARG;
    std::memset(p, 0, sizeof(*p));
    p->struct_size = sizeof(lbm_params);
    p->mode = LBM_MODE_DEFF;
    p->c_in = 1.0;
    p->c_out = 0.0;
    p->tau_ref = 1.0;
    p->w0 = 0.25;
    p->knudsen = 0;
    p->T_K = 353.0;
    p->p_atm = 1.0;
    p->M_kg_mol = 0.032;
    p->d_ionomer_rel = 1e-3;
    p->d_ref_rel = 0.0;
    p->k_lat = 0.0;
    p->catalyst_phases = 1u << LBM_PT;
    p->reactive_fluids = (1u << LBM_PORE) | (1u << LBM_IONOMER);
    p->reservoir_plane = 1;
    p->tol_change = 1e-8;
    p->tol_flux = 1e-5;
    p->tol_balance = 1e-3;
    p->check_every = 1000;
    p->max_steps = 50000000;
    return LBM_OK;
}

int lbm_create(const lbm_grid *g, const uint8_t *phase, const lbm_params *p, lbm_solver **out) {
    LBM_GUARD_BEGIN
    if (!g || !phase || !p || !out) return LBM_ERR_INVALID_ARG;
    *out = nullptr;
    std::unique_ptr<cl::Engine> E;
    const int st = cl::make_engine(1, g, &phase, p, E);
    if (st != LBM_OK) return st;
    auto *s = new lbm_solver;
    s->E = std::move(E);
    *out = s;
    return LBM_OK;
    LBM_GUARD_END
}

int lbm_prep_scratch_bytes(int32_t n, const lbm_grid *grids, const lbm_params *params, size_t *bytes) {
    if (n <= 0 || !grids || !params || !bytes) return LBM_ERR_INVALID_ARG;
    size_t b = 0;
    for (int i = 0; i < n; ++i) {
        if (grids[i].nx <= 0 || grids[i].ny <= 0 || grids[i].nz <= 0) return LBM_ERR_INVALID_ARG;
        b = std::max(b, cl::prep_scratch_bytes(grids[i], params[i]));
    }
    *bytes = b;
    return LBM_OK;
}

// lbm_create / lbm_batch_create with the device share of the preprocessing.
static int create_device(int32_t n, const lbm_grid *grids, const uint8_t *const *phases, const lbm_params *params,
                         void *scratch, size_t bytes, void *stream, std::unique_ptr<cl::Engine> &E) {
    if (!scratch || (reinterpret_cast<uintptr_t>(scratch) & 255)) return LBM_ERR_WORKSPACE;
    if (n <= 0 || n > 65535 || !grids || !phases || !params) return LBM_ERR_INVALID_ARG;
    size_t need = 0;
    for (int i = 0; i < n; ++i) {
        if (grids[i].nx <= 0 || grids[i].ny <= 0 || grids[i].nz <= 0) return LBM_ERR_INVALID_ARG;
        need = std::max(need, cl::prep_scratch_bytes(grids[i], params[i]));
    }
    if (bytes < need) return LBM_ERR_WORKSPACE;  // before any device call
    cl::g_last_error[0] = 0;
    std::mutex mu;
    cl::DeviceAssist d;
    d.scratch = scratch;
    d.bytes = bytes;
    d.stream = stream;
    d.mu = &mu;
    return cl::make_engine(n, grids, phases, params, E, &d);
}

int lbm_create_device(const lbm_grid *g, const uint8_t *phase, const lbm_params *p, void *scratch_dev,
                      size_t scratch_bytes, void *stream, lbm_solver **out) {
    LBM_GUARD_BEGIN
    if (!g || !phase || !p || !out) return LBM_ERR_INVALID_ARG;
    *out = nullptr;
    std::unique_ptr<cl::Engine> E;
    const int st = create_device(1, g, &phase, p, scratch_dev, scratch_bytes, stream, E);
    if (st != LBM_OK) return st;
    auto *s = new lbm_solver;
    s->E = std::move(E);
    *out = s;
    return LBM_OK;
    LBM_GUARD_END
}

int lbm_batch_create_device(int32_t n, const lbm_grid *grids, const uint8_t *const *phases, const lbm_params *params,
                            void *scratch_dev, size_t scratch_bytes, void *stream, lbm_batch **out) {
    LBM_GUARD_BEGIN
    if (!out) return LBM_ERR_INVALID_ARG;
    *out = nullptr;
    std::unique_ptr<cl::Engine> E;
    const int st = create_device(n, grids, phases, params, scratch_dev, scratch_bytes, stream, E);
    if (st != LBM_OK) return st;
    auto *b = new lbm_batch;
    b->E = std::move(E);
    *out = b;
    return LBM_OK;
    LBM_GUARD_END
}

int lbm_get_info(const lbm_solver *s, lbm_info *info) {
    if (!s || !info) return LBM_ERR_INVALID_ARG;
    std::memset(info, 0, sizeof(*info));
    s->E->info_of(0, *info);
    return LBM_OK;
}

int lbm_get_host_fields(const lbm_solver *s, uint8_t *active, uint8_t *n_cat, float *omega) {
    if (!s) return LBM_ERR_INVALID_ARG;
    const cl::Prepared &p = s->E->P[0];
    if (active) std::copy(p.active.begin(), p.active.end(), active);
    if (n_cat) std::copy(p.n_cat.begin(), p.n_cat.end(), n_cat);
    if (omega) std::copy(p.omega_dense.begin(), p.omega_dense.end(), omega);
    return LBM_OK;
}

int lbm_get_pore_depth(const lbm_solver *s, uint8_t *depth) {
    LBM_GUARD_BEGIN
    if (!s || !depth) return LBM_ERR_INVALID_ARG;
    cl::pore_depth(s->E->P[0], depth);
    return LBM_OK;
    LBM_GUARD_END
}

int lbm_workspace_bytes(const lbm_solver *s, size_t *bytes) {
    if (!s || !bytes) return LBM_ERR_INVALID_ARG;
    *bytes = s->E->ws_need;
    return LBM_OK;
}

int lbm_bind(lbm_solver *s, void *ws, size_t bytes, void *stream) {
    LBM_GUARD_BEGIN
    if (!s || !ws) return LBM_ERR_INVALID_ARG;
    if (bytes < s->E->ws_need || (reinterpret_cast<uintptr_t>(ws) % cl::kAlign) != 0) return LBM_ERR_WORKSPACE;
    return cl::hip_status(s->E->bind(ws, bytes, static_cast<hipStream_t>(stream)));
    LBM_GUARD_END
}

int lbm_set_initial_concentration(lbm_solver *s, const float *c_dev) {
    LBM_GUARD_BEGIN
    if (!s) return LBM_ERR_INVALID_ARG;
    if (!s->E->bound) return LBM_ERR_UNBOUND;
    cl::DeviceGuard dg(s->E->device);
    return cl::hip_status(s->E->init(c_dev));
    LBM_GUARD_END
}

int lbm_set_populations(lbm_solver *s, const float *f_dev) {
    if (!s || !f_dev) return LBM_ERR_INVALID_ARG;
    cl::Engine &E = *s->E;
    if (!E.bound) return LBM_ERR_UNBOUND;
    cl::DeviceGuard dg(E.device);
    const int64_t N = (int64_t)E.P[0].nx * E.P[0].ny * E.P[0].nz;
    return cl::hip_status(cl::launch_set_pop(E.L, E.conv_nblk, E.at<int2>(E.off_cblk), f_dev, E.at<int64_t>(E.off_dbase),
                                             N, E.f[E.cur], E.st));
}

int lbm_get_populations(const lbm_solver *s, float *f_dev) {
    if (!s || !f_dev) return LBM_ERR_INVALID_ARG;
    const cl::Engine &E = *s->E;
    if (!E.bound) return LBM_ERR_UNBOUND;
    cl::DeviceGuard dg(E.device);
    const int64_t N = (int64_t)E.P[0].nx * E.P[0].ny * E.P[0].nz;
    hipError_t e = cl::launch_get_pop(E.L, E.conv_nblk, E.at<int2>(E.off_cblk), E.f[E.cur], E.at<int64_t>(E.off_dbase),
                                      N, f_dev, E.st);
    if (e == hipSuccess) e = hipStreamSynchronize(E.st);
    return cl::hip_status(e);
}

int lbm_step(lbm_solver *s, int64_t n) {
    if (!s || n < 0) return LBM_ERR_INVALID_ARG;
    if (!s->E->bound) return LBM_ERR_UNBOUND;
    cl::DeviceGuard dg(s->E->device);
    cl::Engine &E = *s->E;
    hipError_t e = E.all_live();
    if (e == hipSuccess) e = E.steps(n);
    E.rs[0].info.steps += n;
    return cl::hip_status(e);
}

int lbm_measure(lbm_solver *s, lbm_run_info *info) {
    if (!s || !info) return LBM_ERR_INVALID_ARG;
    cl::Engine &E = *s->E;
    if (!E.bound) return LBM_ERR_UNBOUND;
    cl::DeviceGuard dg(E.device);
    hipError_t e = E.all_live();
    if (e == hipSuccess) e = E.measure_enqueue(0);
    if (e == hipSuccess) e = E.read_results();
    if (e != hipSuccess) return LBM_ERR_HIP;
    E.fill_info(0, E.res_host, 0, E.rs[0].info);
    E.rs[0].measured = 1;
    *info = E.rs[0].info;
    return E.res_host[cl::Q_BAD] > 0 ? LBM_ERR_DIVERGED : LBM_OK;
}

int lbm_run_to_steady(lbm_solver *s, lbm_run_info *info) {
    LBM_GUARD_BEGIN
    if (!s) return LBM_ERR_INVALID_ARG;
    cl::DeviceGuard dg(s->E->device);
    cl::Engine &E = *s->E;
    if (!E.bound) return LBM_ERR_UNBOUND;
    E.rs[0].done = 0;
    if (E.all_live() != hipSuccess) return LBM_ERR_HIP;
    lbm_run_info tmp{};
    const int st = E.run(&tmp);
    if (info) *info = tmp;
    return st < 0 ? st : tmp.status;
    LBM_GUARD_END
}

int lbm_advance(lbm_solver *s, int64_t max_new_steps, lbm_run_info *info) {
    LBM_GUARD_BEGIN
    if (!s || max_new_steps < 0) return LBM_ERR_INVALID_ARG;
    cl::DeviceGuard dg(s->E->device);
    cl::Engine &E = *s->E;
    if (!E.bound) return LBM_ERR_UNBOUND;
    E.rs[0].done = 0;
    if (E.all_live() != hipSuccess) return LBM_ERR_HIP;
    lbm_run_info tmp{};
    const int st = E.run(&tmp, max_new_steps);
    if (info) *info = tmp;
    return st < 0 ? st : tmp.status;
    LBM_GUARD_END
}

int lbm_deff(const lbm_solver *s, double *out) {
    if (!s || !out) return LBM_ERR_INVALID_ARG;
    return s->E->deff(0, out);
}

int lbm_reaction_rate(const lbm_solver *s, double *rate, double *jin) {
    if (!s) return LBM_ERR_INVALID_ARG;
    return s->E->rate(0, rate, jin);
}

int lbm_concentration(const lbm_solver *s, float *c_dev) {
    if (!s || !c_dev) return LBM_ERR_INVALID_ARG;
    const cl::Engine &E = *s->E;
    if (!E.bound) return LBM_ERR_UNBOUND;
    cl::DeviceGuard dg(E.device);
    hipError_t e = cl::launch_conc(E.L, E.conv_nblk, E.at<int2>(E.off_cblk), E.react, E.f[E.cur],
                                   E.at<int64_t>(E.off_dbase), c_dev, E.st);
    if (e == hipSuccess) e = hipStreamSynchronize(E.st);
    return cl::hip_status(e);
}

void lbm_destroy(lbm_solver *s) { delete s; }

const char *lbm_last_error(void) { return cl::g_last_error; }

const char *lbm_status_string(int st) {
    switch (st) {
        case LBM_OK: return "ok";
        case LBM_NOT_CONVERGED: return "not converged";
        case LBM_ERR_INVALID_ARG: return "invalid argument";
        case LBM_ERR_BAD_PHASE: return "phase id outside 0..3";
        case LBM_ERR_WRONG_MODE: return "wrong mode for this output";
        case LBM_ERR_NO_PERCOLATION: return "no transport path between the Dirichlet faces";
        case LBM_ERR_DIVERGED: return "diverged (NaN or Inf)";
        case LBM_ERR_HIP: return "HIP runtime error";
        case LBM_ERR_UNBOUND: return "no workspace bound or nothing measured yet";
        case LBM_ERR_WORKSPACE: return "workspace too small or misaligned";
        case LBM_ERR_UNSTABLE: return "unstable parameters (k n >= 1 or tau <= 1/2)";
        default: return "unknown status";
    }
}

// ------------------------------------------------------------------ batched form

int lbm_batch_create(int32_t n, const lbm_grid *grids, const uint8_t *const *phases, const lbm_params *params,
                     lbm_batch **out) {
    LBM_GUARD_BEGIN
    if (!out) return LBM_ERR_INVALID_ARG;
    *out = nullptr;
    std::unique_ptr<cl::Engine> E;
    const int st = cl::make_engine(n, grids, phases, params, E);
    if (st != LBM_OK) return st;
    auto *b = new lbm_batch;
    b->E = std::move(E);
    *out = b;
    return LBM_OK;
    LBM_GUARD_END
}

int lbm_batch_workspace_bytes(const lbm_batch *b, size_t *bytes) {
    if (!b || !bytes) return LBM_ERR_INVALID_ARG;
    *bytes = b->E->ws_need;
    return LBM_OK;
}

int lbm_batch_bind(lbm_batch *b, void *ws, size_t bytes, void *stream) {
    LBM_GUARD_BEGIN
    if (!b || !ws) return LBM_ERR_INVALID_ARG;
    if (bytes < b->E->ws_need || (reinterpret_cast<uintptr_t>(ws) % cl::kAlign) != 0) return LBM_ERR_WORKSPACE;
    return cl::hip_status(b->E->bind(ws, bytes, static_cast<hipStream_t>(stream)));
    LBM_GUARD_END
}

static int set_tiling(cl::Engine &E, int32_t spw, int32_t waves, int32_t xcd) {
    if (!(spw == 1 || spw == 2 || spw == 4) || !(waves == 1 || waves == 2 || waves == 4 || waves == 8))
        return LBM_ERR_INVALID_ARG;
    E.spw = spw;
    E.waves = waves;
    E.xcd = xcd ? 1 : 0;
    if (E.bound) {
        cl::DeviceGuard dg(E.device);
        return cl::hip_status(E.upload_tables());
    }
    return LBM_OK;
}

static int get_tiling(const cl::Engine &E, int32_t *spw, int32_t *waves, int32_t *xcd) {
    if (spw) *spw = E.spw;
    if (waves) *waves = E.waves;
    if (xcd) *xcd = E.xcd;
    return LBM_OK;
}

static int autotune(cl::Engine &E, int32_t steps_per_trial, double *ms_best) {
    LBM_GUARD_BEGIN
    if (steps_per_trial < 2) return LBM_ERR_INVALID_ARG;
    if (E.bound && E.all_live() != hipSuccess) return LBM_ERR_HIP;
    if (!E.bound) return LBM_ERR_UNBOUND;
    cl::DeviceGuard dg(E.device);
    if (steps_per_trial & 1) ++steps_per_trial;  // even: the state stays in its lattice
    // Trial steps are ordinary solver steps: they advance every live instance toward
    // its steady state, so nothing has to be saved or restored.
    hipError_t e = hipSuccess;
    int64_t trial_steps = 0;
    hipEvent_t t0, t1;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) return LBM_ERR_HIP;
    double best = 1e300;
    auto trial = [&]() -> bool {  // times the current form; true if it is the fastest so far
        if ((e = E.upload_tables()) != hipSuccess) return false;
        if ((e = E.steps(2)) != hipSuccess) return false;  // warm-up
        if ((e = hipEventRecord(t0, E.st)) != hipSuccess) return false;
        if ((e = E.steps(steps_per_trial)) != hipSuccess) return false;
        trial_steps += steps_per_trial + 2;
        if ((e = hipEventRecord(t1, E.st)) != hipSuccess) return false;
        if ((e = hipEventSynchronize(t1)) != hipSuccess) return false;
        float ms = 0.f;
        if ((e = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) return false;
        const double per = ms / steps_per_trial;
        if (per >= best) return false;
        best = per;
        return true;
    };
    // one step per launch: segments per wave x waves per workgroup x XCD order
    const int spws[3] = {1, 2, 4};
    const int wavs[4] = {1, 2, 4, 8};
    int bs = E.spw, bw = E.waves, bx = E.xcd, bby = 0, bzc = E.t2_zc;
    E.t2_by = 0;
    for (int xi = 0; xi < 2 && e == hipSuccess; ++xi)
        for (int si = 0; si < 3 && e == hipSuccess; ++si)
            for (int wi = 0; wi < 4 && e == hipSuccess; ++wi) {
                E.spw = spws[si];
                E.waves = wavs[wi];
                E.xcd = xi;
                if (trial()) {
                    bs = E.spw;
                    bw = E.waves;
                    bx = E.xcd;
                }
            }
    // two steps per launch (one instance): rows per tile x planes per chunk x XCD order
    if (E.two_step_possible()) {
        E.spw = bs;
        E.waves = bw;
        const int bys[3] = {4, 6, 8};
        const int zcs[4] = {8, 16, 32, 64};
        for (int xi = 0; xi < 2 && e == hipSuccess; ++xi)
            for (int yi = 0; yi < 3 && e == hipSuccess; ++yi)
                for (int zi = 0; zi < 4 && e == hipSuccess; ++zi) {
                    E.xcd = xi;
                    E.t2_by = bys[yi];
                    E.t2_zc = zcs[zi];
                    if (trial()) {
                        bx = E.xcd;
                        bby = E.t2_by;
                        bzc = E.t2_zc;
                    }
                }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    E.spw = bs;
    E.waves = bw;
    E.xcd = bx;
    E.t2_by = bby;
    E.t2_zc = bzc;
    if (e == hipSuccess) e = E.upload_tables();
    for (int i : E.live) E.rs[i].info.steps += trial_steps;
    if (ms_best) *ms_best = best;
    return cl::hip_status(e);
    LBM_GUARD_END
}

int lbm_batch_set_tiling(lbm_batch *b, int32_t spw, int32_t waves, int32_t xcd) {
    return b ? set_tiling(*b->E, spw, waves, xcd) : LBM_ERR_INVALID_ARG;
}

int lbm_batch_get_tiling(const lbm_batch *b, int32_t *spw, int32_t *waves, int32_t *xcd) {
    return b ? get_tiling(*b->E, spw, waves, xcd) : LBM_ERR_INVALID_ARG;
}

int lbm_batch_autotune(lbm_batch *b, int32_t steps_per_trial, double *ms_best) {
    return b ? autotune(*b->E, steps_per_trial, ms_best) : LBM_ERR_INVALID_ARG;
}

int lbm_set_tiling(lbm_solver *s, int32_t spw, int32_t waves, int32_t xcd) {
    return s ? set_tiling(*s->E, spw, waves, xcd) : LBM_ERR_INVALID_ARG;
}

int lbm_get_tiling(const lbm_solver *s, int32_t *spw, int32_t *waves, int32_t *xcd) {
    return s ? get_tiling(*s->E, spw, waves, xcd) : LBM_ERR_INVALID_ARG;
}

int lbm_set_temporal(lbm_solver *s, int32_t rows_per_tile, int32_t planes_per_chunk) {
    if (!s || !(rows_per_tile == 0 || rows_per_tile == 4 || rows_per_tile == 6 || rows_per_tile == 8))
        return LBM_ERR_INVALID_ARG;
    if (rows_per_tile && (planes_per_chunk < 1 || planes_per_chunk > 64)) return LBM_ERR_INVALID_ARG;
    cl::Engine &E = *s->E;
    if (rows_per_tile && !E.two_step_possible()) return LBM_ERR_INVALID_ARG;
    E.t2_by = rows_per_tile;
    if (rows_per_tile) E.t2_zc = planes_per_chunk;
    E.g_valid = false;  // captured windows hold the previous form
    return LBM_OK;
}

int lbm_get_temporal(const lbm_solver *s, int32_t *rows_per_tile, int32_t *planes_per_chunk) {
    if (!s) return LBM_ERR_INVALID_ARG;
    if (rows_per_tile) *rows_per_tile = s->E->t2_by;
    if (planes_per_chunk) *planes_per_chunk = s->E->t2_zc;
    return LBM_OK;
}

int lbm_autotune(lbm_solver *s, int32_t steps_per_trial, double *ms_best) {
    return s ? autotune(*s->E, steps_per_trial, ms_best) : LBM_ERR_INVALID_ARG;
}

int lbm_batch_run(lbm_batch *b, lbm_run_info *infos) {
    LBM_GUARD_BEGIN
    if (!b) return LBM_ERR_INVALID_ARG;
    cl::DeviceGuard dg(b->E->device);
    return b->E->run_grouped(infos);
    LBM_GUARD_END
}

int lbm_batch_advance(lbm_batch *b, int64_t max_new_steps, lbm_run_info *infos) {
    LBM_GUARD_BEGIN
    if (!b || max_new_steps < 0) return LBM_ERR_INVALID_ARG;
    cl::DeviceGuard dg(b->E->device);
    return b->E->run_grouped(infos, max_new_steps);
    LBM_GUARD_END
}

int lbm_batch_set_group_bytes(lbm_batch *b, int64_t bytes) {
    if (!b || bytes < 0) return LBM_ERR_INVALID_ARG;
    b->E->group_bytes = bytes;
    return LBM_OK;
}

int lbm_batch_deff(const lbm_batch *b, int32_t i, double *out) {
    if (!b || !out || i < 0 || i >= b->E->ninst) return LBM_ERR_INVALID_ARG;
    return b->E->deff(i, out);
}

int lbm_batch_reaction_rate(const lbm_batch *b, int32_t i, double *rate, double *jin) {
    if (!b || i < 0 || i >= b->E->ninst) return LBM_ERR_INVALID_ARG;
    return b->E->rate(i, rate, jin);
}

int lbm_batch_get_info(const lbm_batch *b, int32_t i, lbm_info *info) {
    if (!b || !info || i < 0 || i >= b->E->ninst) return LBM_ERR_INVALID_ARG;
    std::memset(info, 0, sizeof(*info));
    b->E->info_of(i, *info);
    return LBM_OK;
}

int lbm_batch_concentration(const lbm_batch *b, int32_t i, float *c_dev) {
    if (!b || !c_dev || i < 0 || i >= b->E->ninst) return LBM_ERR_INVALID_ARG;
    const cl::Engine &E = *b->E;
    if (!E.bound) return LBM_ERR_UNBOUND;
    cl::DeviceGuard dg(E.device);
    hipError_t e = cl::launch_conc(E.L, E.cb_count[i], E.at<int2>(E.off_cblk) + E.cb_start[i], E.react, E.f[E.cur],
                                   E.at<int64_t>(E.off_zbase), c_dev, E.st);
    if (e == hipSuccess) e = hipStreamSynchronize(E.st);
    return cl::hip_status(e);
}

int lbm_batch_get_host_fields(const lbm_batch *b, int32_t i, uint8_t *active, uint8_t *n_cat, float *omega) {
    if (!b || i < 0 || i >= b->E->ninst) return LBM_ERR_INVALID_ARG;
    const cl::Prepared &p = b->E->P[i];
    if (active) std::copy(p.active.begin(), p.active.end(), active);
    if (n_cat) std::copy(p.n_cat.begin(), p.n_cat.end(), n_cat);
    if (omega) std::copy(p.omega_dense.begin(), p.omega_dense.end(), omega);
    return LBM_OK;
}

int lbm_batch_get_pore_depth(const lbm_batch *b, int32_t i, uint8_t *depth) {
    LBM_GUARD_BEGIN
    if (!b || !depth || i < 0 || i >= b->E->ninst) return LBM_ERR_INVALID_ARG;
    cl::pore_depth(b->E->P[i], depth);
    return LBM_OK;
    LBM_GUARD_END
}

void lbm_batch_destroy(lbm_batch *b) { delete b; }

}  // extern "C"
