// Structure characterisation on the device (Chen et al., arXiv 1410.1914,
// Section 2.1.3): the 13-direction pore size behind the Knudsen diffusivity
// (Eqs. 8-9), and the reach of the transport phases from the Dirichlet faces.
// These are the two host steps of lbm_create whose cost grows with the voxel
// count; here they run on maps already resident in HBM.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <numeric>

#include "kernels.h"
#include "prep.h"

namespace {

// The 13 directions of Section 2.1.3 (one of each opposite pair), in the order in
// which their contributions are summed, with |d| and, for directions without an
// x component, the number of voxels on their closed loop under the y/z wrap.
struct Dir13 {
    int d[13][3];
    double len[13];
    int64_t cap[13];
};

constexpr int kDirs[13][3] = {{1, 0, 0},  {0, 1, 0},  {0, 0, 1}, {1, 1, 0},  {1, -1, 0}, {1, 0, 1},  {1, 0, -1},
                              {0, 1, 1},  {0, 1, -1}, {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {-1, 1, 1}};

__device__ __forceinline__ int wrap1(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// Pore size of every voxel: for each direction, the run of pore voxels through it
// (walked both ways, bounded by the x faces, at most one loop when the line closes
// on itself), times |d|; the mean over the 13 directions.  The products and sums
// are kept apart (no fused multiply-add), as in a plain FP64 evaluation.
__global__ __launch_bounds__(256) void k_pore_size(const uint8_t *__restrict__ pore, int nx, int ny, int nz, Dir13 D,
                                                   double *__restrict__ dp) {
    const int64_t N = (int64_t)nx * ny * nz;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    if (!pore[v]) {
        dp[v] = 0.0;
        return;
    }
    const int x = (int)(v % nx);
    const int64_t row = v / nx;
    const int y = (int)(row % ny), z = (int)(row / ny);
    double sum = 0.0;
    for (int d = 0; d < 13; ++d) {
        const int dx = D.d[d][0], dy = D.d[d][1], dz = D.d[d][2];
        const int64_t cap = D.cap[d];
        int64_t count = 1;
        for (int s = -1; s <= 1; s += 2) {
            int cx = x, cy = y, cz = z;
            while (count < cap) {
                cx += s * dx;
                cy = wrap1(cy + s * dy, ny);
                cz = wrap1(cz + s * dz, nz);
                if (cx < 0 || cx >= nx) break;
                if (!pore[((int64_t)cz * ny + cy) * nx + cx]) break;
                ++count;
            }
        }
        {
#pragma clang fp contract(off)
            sum = sum + (double)count * D.len[d];
        }
    }
    dp[v] = sum / 13.0;
}

// Seeds of the reach: pass voxels on the selected x faces.
__global__ __launch_bounds__(256) void k_reach_seed(const uint8_t *__restrict__ pass, int nx, int ny, int nz, int faces,
                                                    uint8_t *__restrict__ hit) {
    const int64_t N = (int64_t)nx * ny * nz;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    const int x = (int)(v % nx);
    hit[v] = (uint8_t)(pass[v] && (((faces & 1) && x == 0) || ((faces & 2) && x == nx - 1)));
}

// One sweep along `axis` (0 x, 1 y, 2 z): one thread per line, walked forward and
// then backward, carrying reach along the line and taking it from the four
// neighbours across the line.  Reach only ever turns on, so threads racing on a
// voxel agree; a sweep that turns nothing on leaves *changed untouched.
__global__ __launch_bounds__(256) void k_reach_sweep(const uint8_t *__restrict__ pass, uint8_t *hit, int nx, int ny,
                                                     int nz, int axis, int *changed) {
    const int n[3] = {nx, ny, nz};
    const int a1 = axis == 0 ? 1 : 0, a2 = axis == 2 ? 1 : 2;  // the two axes across the line
    const int64_t lines = (int64_t)n[a1] * n[a2];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= lines) return;
    int c[3];
    c[a1] = (int)(t % n[a1]);
    c[a2] = (int)(t / n[a1]);
    const int L = n[axis];
    auto at = [&](int cx, int cy, int cz) { return ((int64_t)cz * ny + cy) * nx + cx; };
    auto across = [&](int i) -> bool {  // reach of a neighbour across the line, with the y/z wrap
        int p[3] = {c[0], c[1], c[2]};
        p[axis] = i;
        const int cx = p[0], cy = p[1], cz = p[2];
        bool h = false;
        if (axis != 0) {
            if (cx > 0) h = h || hit[at(cx - 1, cy, cz)];
            if (cx + 1 < nx) h = h || hit[at(cx + 1, cy, cz)];
        }
        if (axis != 1) h = h || hit[at(cx, wrap1(cy - 1, ny), cz)] || hit[at(cx, wrap1(cy + 1, ny), cz)];
        if (axis != 2) h = h || hit[at(cx, cy, wrap1(cz - 1, nz))] || hit[at(cx, cy, wrap1(cz + 1, nz))];
        return h;
    };
    bool any = false;
    for (int pass_dir = 0; pass_dir < 2; ++pass_dir) {
        bool carry = false;
        for (int k = 0; k < L; ++k) {
            const int i = pass_dir ? L - 1 - k : k;
            int p[3] = {c[0], c[1], c[2]};
            p[axis] = i;
            const int64_t v = at(p[0], p[1], p[2]);
            if (!pass[v]) {
                carry = false;
                continue;
            }
            bool h = hit[v] != 0;
            if (!h && (carry || across(i))) {
                hit[v] = 1;
                h = true;
                any = true;
            }
            carry = h;
        }
    }
    if (any) *changed = 1;
}

// Bits of p in a run (maximal block of consecutive set bits) that holds a bit of
// h (h within p): adding h to p carries from the lowest such bit to the run's end,
// the same on reversed bits covers the run's start.
__device__ __forceinline__ uint64_t fill_runs(uint64_t p, uint64_t h) {
    const uint64_t up = ((p + h) ^ p) & p;
    const uint64_t pr = __brevll(p), hr = __brevll(h);
    const uint64_t down = __brevll(((pr + hr) ^ pr) & pr);
    return up | down | h;
}

// The x sweep with one wave per x line: 64 voxels at a time as bit masks (pass,
// reach including the four neighbours across the line), runs filled with
// fill_runs, and reach carried across 64-voxel chunks forward and then backward.
__global__ __launch_bounds__(256) void k_reach_sweep_x(const uint8_t *__restrict__ pass, uint8_t *hit, int nx,
                                                       int ny, int nz, int *changed) {
    const int lane = threadIdx.x & 63;
    const int64_t line = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (line >= (int64_t)ny * nz) return;  // whole waves leave together
    const int y = (int)(line % ny), z = (int)(line / ny);
    const int64_t base = line * nx;
    const int64_t ym = ((int64_t)z * ny + wrap1(y - 1, ny)) * nx, yp = ((int64_t)z * ny + wrap1(y + 1, ny)) * nx;
    const int64_t zm = ((int64_t)wrap1(z - 1, nz) * ny + y) * nx, zp = ((int64_t)wrap1(z + 1, nz) * ny + y) * nx;
    const int nch = (nx + 63) / 64;
    bool any = false;
    for (int dir = 0; dir < 2; ++dir) {
        bool carry = false;  // the voxel next to this chunk, on the side already swept, is reached
        for (int k = 0; k < nch; ++k) {
            const int c = dir ? nch - 1 - k : k;
            const int x = c * 64 + lane;
            const bool in = x < nx;
            const bool ps = in && pass[base + x];
            const bool h0 = ps && hit[base + x];
            const bool ac = ps && (hit[ym + x] || hit[yp + x] || hit[zm + x] || hit[zp + x]);
            const uint64_t P = __ballot(ps);
            uint64_t H = __ballot(h0 || ac);
            if (carry) H |= dir ? (P & (1ull << 63)) : (P & 1ull);
            const uint64_t R = P ? fill_runs(P, H) : 0ull;
            const bool now = (R >> lane) & 1ull;
            if (now && !h0) {
                hit[base + x] = 1;
                any = true;
            }
            const int edge = dir ? 0 : 63;  // the chunk's last voxel in sweep order
            carry = ((R >> edge) & 1ull) != 0 && (dir ? c * 64 : c * 64 + 63) < nx;
        }
    }
    if (any) *changed = 1;
}

// Clears n counters of the allocation-free reach's scratch (a kernel, not a
// memset, so the call stays free of memset nodes if a caller ever records it).
__global__ void k_zero_i32(int32_t *p, int n) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) p[i] = 0;
}

}  // namespace

// Scratch of lbm_reach_device_static: counters in device memory that the library
// never allocates.  Slot 0 is the change flag of the current sweep cycle; the rest
// is reserved.  Each device holds its own copy for the life of the process.
constexpr int kReachScratchInts = 64;  // 256 bytes
static __device__ __align__(256) int32_t scratch[kReachScratchInts];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t *g_scratch_dev[kMaxDevices];  // device address of `scratch`, per device

// The device address of this device's `scratch`, looked up once per device with
// that device current (the symbol's host-side name is not a device address).
hipError_t reach_scratch(int32_t **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = static_cast<int32_t *>(ptr);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

// Seeds, then sweep cycles until one turns nothing on: the loop both reach entry
// points share.  `flag_dev` is the change flag the sweeps set; flag(true, nullptr)
// clears it before a cycle, flag(false, &v) waits for the cycle's work and reads
// it into v.
template <class Flag>
hipError_t reach_cycles(const uint8_t *pass_dev, int32_t nx, int32_t ny, int32_t nz, int32_t faces, uint8_t *hit_dev,
                        hipStream_t st, int32_t *flag_dev, Flag &&flag, int32_t *n_cycles) {
    const int64_t N = (int64_t)nx * ny * nz;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_reach_seed, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, pass_dev, nx, ny, nz, faces,
                       hit_dev);
    hipError_t e = hipGetLastError();
    *n_cycles = 0;
    // every productive cycle turns at least one voxel on, so at most N + 1 cycles run
    for (int64_t cyc = 0; e == hipSuccess && cyc <= N; ++cyc) {
        e = flag(true, nullptr);
        if (e != hipSuccess) break;
        {
            const int64_t lines = (int64_t)ny * nz;  // x: one wave per line
            hipLaunchKernelGGL(k_reach_sweep_x, dim3((unsigned)((lines + 3) / 4)), dim3(256), 0, st, pass_dev, hit_dev,
                               nx, ny, nz, flag_dev);
            e = hipGetLastError();
        }
        for (int axis = 1; axis < 3 && e == hipSuccess; ++axis) {  // y, z: one thread per line
            const int64_t lines = axis == 1 ? (int64_t)nx * nz : (int64_t)nx * ny;
            hipLaunchKernelGGL(k_reach_sweep, dim3((unsigned)((lines + 255) / 256)), dim3(256), 0, st, pass_dev, hit_dev,
                               nx, ny, nz, axis, flag_dev);
            e = hipGetLastError();
        }
        int32_t changed = 0;
        if (e == hipSuccess) e = flag(false, &changed);
        ++*n_cycles;
        if (e != hipSuccess || !changed) break;
    }
    return e;
}

}  // namespace

extern "C" {

int lbm_pore_size_device(const uint8_t *pore_dev, int32_t nx, int32_t ny, int32_t nz, double *dp_dev, void *stream) {
    if (!pore_dev || !dp_dev || nx <= 0 || ny <= 0 || nz <= 0) return LBM_ERR_INVALID_ARG;
    const int64_t N = (int64_t)nx * ny * nz;
    if ((N + 255) / 256 > INT32_MAX) return LBM_ERR_INVALID_ARG;
    Dir13 D{};
    for (int d = 0; d < 13; ++d) {
        const int dx = kDirs[d][0], dy = kDirs[d][1], dz = kDirs[d][2];
        for (int k = 0; k < 3; ++k) D.d[d][k] = kDirs[d][k];
        D.len[d] = std::sqrt((double)(dx * dx + dy * dy + dz * dz));
        D.cap[d] = dx != 0 ? INT64_MAX : (dy != 0 && dz != 0 ? std::lcm((int64_t)ny, (int64_t)nz) : (dy ? ny : nz));
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_pore_size, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, pore_dev, nx, ny, nz, D, dp_dev);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return cl::record_error(e, "lbm_pore_size_device");
}

int lbm_reach_device(const uint8_t *pass_dev, int32_t nx, int32_t ny, int32_t nz, int32_t faces, uint8_t *hit_dev,
                     int32_t *cycles, void *stream) {
    if (!pass_dev || !hit_dev || nx <= 0 || ny <= 0 || nz <= 0 || faces < 1 || faces > 3) return LBM_ERR_INVALID_ARG;
    const int64_t N = (int64_t)nx * ny * nz;
    if ((N + 255) / 256 > INT32_MAX) return LBM_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int *changed = nullptr;  // one flag, in pinned host memory the device writes directly
    hipError_t e = hipHostMalloc((void **)&changed, sizeof(int), hipHostMallocMapped);
    int *changed_dev = nullptr;
    if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&changed_dev, changed, 0);
    int32_t n_cycles = 0;
    if (e == hipSuccess) {
        auto flag = [&](bool zero, int32_t *value) -> hipError_t {
            if (zero) {
                *changed = 0;
                return hipSuccess;
            }
            const hipError_t se = hipStreamSynchronize(st);
            *value = *changed;
            return se;
        };
        e = reach_cycles(pass_dev, nx, ny, nz, faces, hit_dev, st, changed_dev, flag, &n_cycles);
    }
    if (changed) (void)hipHostFree(changed);
    if (cycles) *cycles = n_cycles;
    return cl::record_error(e, "lbm_reach_device");
}

int lbm_reach_device_static(const uint8_t *pass_dev, int32_t nx, int32_t ny, int32_t nz, int32_t faces,
                            uint8_t *hit_dev, int32_t *cycles, void *stream) {
    if (!pass_dev || !hit_dev || nx <= 0 || ny <= 0 || nz <= 0 || faces < 1 || faces > 3) return LBM_ERR_INVALID_ARG;
    const int64_t N = (int64_t)nx * ny * nz;
    if ((N + 255) / 256 > INT32_MAX) return LBM_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int32_t *flag_dev = nullptr;
    hipError_t e = reach_scratch(&flag_dev);
    int32_t n_cycles = 0;
    if (e == hipSuccess) {
        auto flag = [&](bool zero, int32_t *value) -> hipError_t {
            if (zero) {
                hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, flag_dev, 1);
                return hipGetLastError();
            }
            hipError_t ce = hipMemcpyAsync(value, flag_dev, sizeof(int32_t), hipMemcpyDeviceToHost, st);
            if (ce == hipSuccess) ce = hipStreamSynchronize(st);
            return ce;
        };
        e = reach_cycles(pass_dev, nx, ny, nz, faces, hit_dev, st, flag_dev, flag, &n_cycles);
    }
    if (cycles) *cycles = n_cycles;
    return cl::record_error(e, "lbm_reach_device_static");
}

}  // extern "C"
