// Kernels of the learned warm start's 3-D U-Net (gfx950): BF16 MFMA implicit-GEMM
// 3x3x3 convolutions with FP32 accumulation, their backward passes, pooling,
// upsampling, the output head, the masked MSE loss and Adam.  The C ABI is in
// include/unet.h.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <algorithm>

#include "../../include/unet.h"

namespace {

typedef __bf16 bf16x8 __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef float f32x4 __attribute__((__vector_size__(4 * sizeof(float))));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__host__ __device__ __forceinline__ int kpad_of(int cin) { return (27 * cin + 31) / 32 * 32; }

int status(hipError_t e) { return e == hipSuccess ? 0 : -6; }

// ------------------------------------------------------------------ conv3d forward
//
// Implicit GEMM: rows = voxels, columns = output channels, K = 27 taps x cin, on
// v_mfma_f32_16x16x32_bf16.  Fragment mapping (pinned by unet_mfma_selftest):
//   A[m][k]: lane l holds m = l % 16, k = 8 (l / 16) + j;  B[k][n]: n = l % 16, same k;
//   D[m][n]: lane l holds m = 4 (l / 16) + i, n = l % 16.
// A workgroup (4 waves) owns kTY rows of kTX voxels in ZC consecutive planes and
// 16 * NT output channels (a channel slice).  Per stage of 16 input channels it
// copies the ZC + 2 input planes its planes read ((kTY + 2) rows x
// (kTX + 2) voxels each, halo included) straight from global memory into LDS, all
// in flight at once and with no registers in between, so each input plane is copied
// once per stage rather than once for every output plane that reads it.  Each
// wave takes one row: per K chunk of 32 (two taps of the 16 channels) it reads four
// input fragments from LDS (four 16-voxel tiles), holds NT weight fragments (the
// same for every wave) and issues 4 x NT MFMAs, so an input fragment feeds NT
// products and a weight fragment four.  The weights are the MFMA's A operand and
// the inputs its B operand, so a lane's result is four consecutive output channels
// of one voxel, which leave as one 8-byte store.
struct ConvArgs {
    const uint16_t *x;
    const uint16_t *w;
    const float *b;
    uint16_t *y;
    float *y32;
    int ldx, offx, ldy, offy;
    int nz, ny, nx, cin, cout, kpad, relu;
    uint32_t xbytes, plane_bytes;  // bytes of x and of one of its planes
    uint32_t wbytes;               // bytes of w
    // Input channels [cin1, cin) come from x2 instead (the concatenation of a skip
    // tensor and an upsampled one, never stored): rows of ldx2 at offset offx2, at
    // half resolution in every direction when up2 (nearest upsampling).
    const uint16_t *x2;
    int ldx2, offx2, cin1, up2;
    uint32_t x2bytes, plane2_bytes;
    // The network's 1x1x1 head fused into the last convolution (z-marching form,
    // 16 channels): hout[v] = hb + hbase[v] + sum_c hw[c] y[v, c] on the BF16 outputs,
    // which are then not stored.
    const float *hw, *hb, *hbase;
    float *hout;
};

typedef __attribute__((address_space(3))) void lds_void;

// dword 3 of a raw (untyped, unswizzled) buffer resource on the gfx9 family
constexpr int kRawBuffer = 0x00020000;
// Input planes and weights are read through buffer resources with 32-bit offsets:
// x and w stay below 2 GiB so that kNoOff lies past their ends, and a load at kNoOff
// returns zeros (the staged entries outside the grid, the weights past the 27th tap).
constexpr int64_t kMaxX = ((int64_t)1 << 31) - 16;
constexpr uint32_t kNoOff = 0x80000000u;

constexpr int kTX = 64, kTY = 4;            // voxels of a workgroup in each of its planes: 4 rows of 64
constexpr int kBX = kTX + 2, kBY = kTY + 2; // an input plane, halo included
constexpr int kPlane = kBX * kBY;           // 396 voxels
constexpr int kCC = 16;                     // input channels per stage
constexpr int kVS = 16;  // LDS elements per voxel: the 16 channels, unpadded.  A 32-byte voxel
                         // stride reads at the full LDS rate on gfx950 (the lanes' 16-byte
                         // reads tile whole 512-byte spans); a padded 48-byte stride ran 1.5x slower
constexpr int kKC = 14;  // K chunks of 32 per stage: 27 taps x 16 channels, the last half empty
constexpr int kPS = (2 * kPlane + 255) / 256;  // 16-byte loads per thread and input plane

// ZC output planes per workgroup: the accumulators of ZC planes and the stage's
// weight fragments stay in registers (218 VGPRs at ZC = 3, 256 at ZC = 4; two
// workgroups per CU, 63 or 76 KB of LDS each).  A tile re-reads (ZC + 2) / ZC of its
// input planes, and each stage's loads are exposed once per ZC planes, so larger
// grids take ZC = 4; small ones keep ZC = 3 for more workgroups.
constexpr int kZcLargeGrid = 2048;  // workgroups at ZC = 4 from which ZC = 4 is used
constexpr int kZmWorkgroups = 1536; // the z-marching form aims for about this many workgroups
// s_waitcnt vmcnt(0) (expcnt and lgkmcnt at their maxima: not waited for) on gfx9
constexpr int kWaitVmcnt0 = 0x0F70;

// The tile of this workgroup: x and y origin, plane chunk and channel slice.  The grid
// is (x-y tiles, plane chunks, channel slices).  Workgroups reach the 8 XCDs
// round-robin by launch index b; XCD b % 8 takes a contiguous eighth of the tile
// order, so that tiles sharing input rows and planes run together under one L2 (the
// input copies are the convolution's bottleneck).  Within a channel slice the tiles go
// in bands of four tile rows in y: x fastest, then y within the band, then the plane
// chunks, then the bands (the last band may be shorter).
struct ConvTile {
    int x0, y0, zc, slice;
};
__device__ __forceinline__ ConvTile conv_tile(int nx) {
    const int nxt = (nx + kTX - 1) / kTX;
    const int nblk = (int)(gridDim.x * gridDim.y * gridDim.z);
    const int b = (int)(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z));
    const int xcd = b % 8, per = nblk / 8, extra = nblk % 8;
    const int t = xcd * per + min(xcd, extra) + b / 8;
    constexpr int kYB = 4;
    const int nyt = (int)gridDim.x / nxt, nzc = (int)gridDim.y;
    const int per_slice = (int)gridDim.x * nzc;
    const int slice = t / per_slice, rem = t % per_slice;
    const int band = rem / (nxt * kYB * nzc), in_band = rem % (nxt * kYB * nzc);
    const int h = min(kYB, nyt - band * kYB);
    const int xt = in_band % nxt, yin = (in_band / nxt) % h, zc = in_band / (nxt * h);
    return ConvTile{xt * kTX, (band * kYB + yin) * kTY, zc, slice};
}

template <int NT, int ZC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_conv_fwd(ConvArgs a) {
    __shared__ __attribute__((aligned(16))) uint16_t slab[(ZC + 2) * kPlane * kVS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // each tile reads 5/3 x 6/4 of its own input (ZC = 3)
    const ConvTile T = conv_tile(a.nx);
    const int x0 = T.x0, y0 = T.y0;
    const int z0 = T.zc * ZC;
    const int co0 = T.slice * 16 * NT;
    const int m = lane & 15, kb = lane >> 4;
    f32x4 acc[ZC][4][NT];
#pragma unroll
    for (int p = 0; p < ZC; ++p)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int n = 0; n < NT; ++n) acc[p][t][n] = (f32x4){0.f, 0.f, 0.f, 0.f};
    // this lane's two taps per K chunk: tap = 2 q + (kb >> 1), channels 8 (kb & 1) .. + 7
    const int chan = 8 * (kb & 1);
    // weights through a buffer resource: this lane's byte offset of output channel
    // co0 + 16 n + m, its tap parity kb >> 1 and channel half; the chunk's part is uniform
    const __amdgpu_buffer_rsrc_t rw =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t *>(a.w), (short)0, (int)a.wbytes, kRawBuffer);
    uint32_t woff[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) woff[n] = 2u * (uint32_t)((co0 + 16 * n + m) * a.kpad + (kb >> 1) * a.cin + chan);
    // One input plane straight from global memory into slot `slot` of the LDS slab:
    // 16 bytes per lane, lanes landing on consecutive 16-byte LDS entries (voxel-major,
    // two entries per voxel).  poff: this thread's byte offsets within a plane of the
    // stage's source, or kNoOff outside the grid.
    const __amdgpu_buffer_rsrc_t rx =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t *>(a.x), (short)0, (int)a.xbytes, kRawBuffer);
    const __amdgpu_buffer_rsrc_t rx2 =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t *>(a.x2), (short)0, (int)a.x2bytes, kRawBuffer);
    uint32_t poff[kPS];
    auto source_offsets = [&](bool second) {
        const int sh = second && a.up2 ? 1 : 0, ld = second ? a.ldx2 : a.ldx, off = second ? a.offx2 : a.offx;
#pragma unroll
        for (int it = 0; it < kPS; ++it) {
            const int e = tid + 256 * it, bv = e >> 1, h = e & 1;
            const int xx = x0 + bv % kBX - 1, yy = y0 + bv / kBX - 1;
            const bool in = xx >= 0 && xx < a.nx && yy >= 0 && yy < a.ny;
            poff[it] = in ? 2u * (uint32_t)(((yy >> sh) * (a.nx >> sh) + (xx >> sh)) * ld + off + 8 * h) : kNoOff;
        }
    };
    auto dma_plane = [&](int zz, int c0, int slot) {
        const bool second = c0 >= a.cin1;
        const bool zin = zz >= 0 && zz < a.nz;  // else the whole plane reads as zeros
        const uint32_t zoff = !zin ? 0u
                              : second ? (uint32_t)(a.up2 ? zz >> 1 : zz) * a.plane2_bytes + 2u * (uint32_t)(c0 - a.cin1)
                                       : (uint32_t)zz * a.plane_bytes + 2u * (uint32_t)c0;
#pragma unroll
        for (int it = 0; it < kPS; ++it) {
            const int e0 = 256 * it + 64 * wave, e = e0 + lane;
            if (e0 >= 2 * kPlane) break;  // wave-uniform
            if (e < 2 * kPlane)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(second ? rx2 : rx,
                                                         (lds_void *)(slab + (slot * kPlane * kVS + 8 * e0)), 16,
                                                         zin ? poff[it] : kNoOff, zoff, 0, 0);
        }
    };
    for (int c0 = 0; c0 < a.cin; c0 += kCC) {
        if (c0 == 0 || c0 == a.cin1) source_offsets(c0 >= a.cin1);
        __syncthreads();  // the previous stage's reads of the slab are done
        // every input plane of the stage in flight at once (plane z0 - 1 + s in slot s),
        // and with them the stage's weight fragments: K chunk q, output tile n (zero
        // past the 27th tap)
#pragma unroll
        for (int s = 0; s < ZC + 2; ++s) dma_plane(z0 - 1 + s, c0, s);
        bf16x8 B[kKC][NT];
#pragma unroll
        for (int q = 0; q < kKC; ++q) {
            const int tap = 2 * q + (kb >> 1);
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                // past the 27th tap the offset lies past w: zeros
                const uint32_t vo = tap < 27 ? woff[n] : kNoOff;
                B[q][n] = __builtin_bit_cast(
                    bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rw, vo, 2u * (uint32_t)(2 * q * a.cin + c0), 0));
            }
        }
        __syncthreads();  // waits for the copies (vmcnt) and publishes them
#pragma unroll
        for (int p = 0; p < ZC; ++p) {
            // A fragments of K chunk q from the slab (zero past the 27th tap)
            auto read_a = [&](int q, bf16x8(&A)[4]) {
                const int tap = 2 * q + (kb >> 1);
                const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;  // dz 0..2 from the output plane's slot
                const int base = (p + dz) * kPlane + (wave + dy) * kBX + m + dx;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    uint4 av = make_uint4(0u, 0u, 0u, 0u);
                    if (tap < 27) av = *reinterpret_cast<const uint4 *>(&slab[(base + 16 * t) * kVS + chan]);
                    A[t] = __builtin_bit_cast(bf16x8, av);
                }
            };
            // one K chunk ahead, into the other of two fragment sets (chunk parity, no
            // copies): the next chunk's LDS reads run under this chunk's products
            bf16x8 Af[2][4];
            read_a(0, Af[0]);
#pragma unroll
            for (int q = 0; q < kKC; ++q) {
                if (q + 1 < kKC) read_a(q + 1, Af[(q + 1) & 1]);
                __builtin_amdgcn_sched_barrier(0);  // the reads go out ahead of the products
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int n = 0; n < NT; ++n)
                        acc[p][t][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(B[q][n], Af[q & 1][t], acc[p][t][n], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);  // keep later chunks' reads out of this one
            }
        }
    }
    // Epilogue: with the weights as the A operand each lane holds four consecutive
    // output channels of one voxel, stored as one 8-byte run (16 bytes for FP32)
    const int yy = y0 + wave;
    if (yy >= a.ny) return;
#pragma unroll
    for (int p = 0; p < ZC; ++p) {
        const int zz = z0 + p;
        if (zz >= a.nz) break;
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int c = co0 + 16 * n + 4 * kb;
            float bias[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) bias[i] = a.b ? a.b[c + i] : 0.f;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int xx = x0 + 16 * t + m;
                if (xx >= a.nx) continue;
                const int64_t vm = ((int64_t)zz * a.ny + yy) * a.nx + xx;
                float v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    v[i] = acc[p][t][n][i] + bias[i];
                    if (a.relu) v[i] = fmaxf(v[i], 0.f);
                }
                const uint2 o = make_uint2((uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16),
                                           (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16));
                *reinterpret_cast<uint2 *>(a.y + vm * a.ldy + a.offy + c) = o;
                if (a.y32) *reinterpret_cast<float4 *>(a.y32 + vm * a.cout + c) = make_float4(v[0], v[1], v[2], v[3]);
            }
        }
    }
}

// Single-stage form for 16 input channels: a workgroup marches through a run of zr
// output planes of its 4 x 64 tile.  Input plane z0 - 1 + i lives in ring slot i & 3
// (four distinct LDS arrays, chosen at compile time by a loop unrolled four times);
// while output plane p is computed from slots p, p + 1, p + 2, input plane z0 + p + 2
// is copied straight into slot p + 3, so each plane is copied once per run and the
// copy runs under the products (the compiler keeps a read of one slot from waiting
// on the copy into another only while every read names its slot at compile time).
// A plane's BF16 results are stored at the next step, after that step's copy is
// issued, so a barrier (which waits for the copies) never waits for fresh stores.
// One plane of accumulators, 240 VGPRs: two workgroups per CU.  HEAD: the head is
// applied in the epilogue and only its FP32 output is stored.
template <bool HEAD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_conv_zm(ConvArgs a, int zr) {
    __shared__ __attribute__((aligned(16))) uint16_t s0[kPlane * kVS], s1[kPlane * kVS], s2[kPlane * kVS],
        s3[kPlane * kVS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const ConvTile T = conv_tile(a.nx);
    const int x0 = T.x0, y0 = T.y0;
    const int z0 = T.zc * zr, co0 = T.slice * 16;
    const int n = min(zr, a.nz - z0);  // output planes of this run, at least one
    const int m = lane & 15, kb = lane >> 4, chan = 8 * (kb & 1);
    const int yy = y0 + wave, c = co0 + 4 * kb;
    // weights (once: a single stage) and biases
    const __amdgpu_buffer_rsrc_t rw =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t *>(a.w), (short)0, (int)a.wbytes, kRawBuffer);
    const uint32_t woff = 2u * (uint32_t)((co0 + m) * a.kpad + (kb >> 1) * a.cin + chan);
    bf16x8 B[kKC];
#pragma unroll
    for (int q = 0; q < kKC; ++q) {
        const int tap = 2 * q + (kb >> 1);
        B[q] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rw, tap < 27 ? woff : kNoOff,
                                                                                  2u * (uint32_t)(2 * q * a.cin), 0));
    }
    float bias[4], hw[4], hb = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        bias[i] = a.b ? a.b[c + i] : 0.f;
        hw[i] = HEAD ? a.hw[c + i] : 0.f;
    }
    if (HEAD) hb = a.hb[0];
    const __amdgpu_buffer_rsrc_t rx =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t *>(a.x), (short)0, (int)a.xbytes, kRawBuffer);
    uint32_t poff[kPS];
#pragma unroll
    for (int it = 0; it < kPS; ++it) {
        const int e = tid + 256 * it, bv = e >> 1, h = e & 1;
        const int xx = x0 + bv % kBX - 1, yq = y0 + bv / kBX - 1;
        const bool in = xx >= 0 && xx < a.nx && yq >= 0 && yq < a.ny;
        poff[it] = in ? 2u * (uint32_t)((yq * a.nx + xx) * a.ldx + a.offx + 8 * h) : kNoOff;
    }
    auto copy_plane = [&](int zz, uint16_t *slot) __attribute__((always_inline)) {
        const bool zin = zz >= 0 && zz < a.nz;  // else the plane reads as zeros
        const uint32_t zoff = zin ? (uint32_t)zz * a.plane_bytes : 0u;
#pragma unroll
        for (int it = 0; it < kPS; ++it) {
            const int e0 = 256 * it + 64 * wave, e = e0 + lane;
            if (e0 >= 2 * kPlane) break;  // wave-uniform
            if (e < 2 * kPlane)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, (lds_void *)(slot + 8 * e0), 16, zin ? poff[it] : kNoOff,
                                                         zoff, 0, 0);
        }
    };
    // BF16 results of the previous plane, stored after the next copy is issued (the
    // FP32 results, written in training only, leave at once)
    uint2 pend0 = make_uint2(0u, 0u), pend1 = pend0, pend2 = pend0, pend3 = pend0;
    float hpend0 = 0.f, hpend1 = 0.f, hpend2 = 0.f, hpend3 = 0.f;  // HEAD: the head's outputs
    int pend_z = -1;
    auto flush = [&]() __attribute__((always_inline)) {
        const bool row = pend_z >= 0 && yy < a.ny;
#pragma unroll
        for (int t4 = 0; t4 < 4; ++t4) {
            const int xx = x0 + 16 * t4 + m;
            if (row && xx < a.nx) {
                const int64_t vm = ((int64_t)pend_z * a.ny + yy) * a.nx + xx;
                if (HEAD) {
                    if (kb == 3) a.hout[vm] = t4 == 0 ? hpend0 : t4 == 1 ? hpend1 : t4 == 2 ? hpend2 : hpend3;
                } else {
                    *reinterpret_cast<uint2 *>(a.y + vm * a.ldy + a.offy + c) =
                        t4 == 0 ? pend0 : t4 == 1 ? pend1 : t4 == 2 ? pend2 : pend3;
                }
            }
        }
    };
    // Output plane z0 + p reads the slots of input planes z0 + p - 1 .. z0 + p + 1
    // (ring slots p, p + 1, p + 2, mod 4) while input plane z0 + p + 2 is copied into
    // slot p + 3; the loop runs four planes per trip so that every slot is a fixed
    // array in each of them.  ring(i): slot i, a constant once the loop is unrolled.
    auto ring = [&](int i) -> uint16_t * {
        i &= 3;
        return i == 0 ? s0 : i == 1 ? s1 : i == 2 ? s2 : s3;
    };
    copy_plane(z0 - 1, s0);
    copy_plane(z0, s1);
    copy_plane(z0 + 1, s2);
    for (int p0 = 0; p0 < n; p0 += 4) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int p = p0 + k;
            if (p >= n) break;
            // This plane's inputs have landed (each wave waits for its own copies, the
            // barrier for all of them) and every wave is done with slot k + 3's plane.
            // The wait is explicit: the compiler does not carry the copy issued in the
            // last step of a trip around the loop's back edge.
            __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
            __syncthreads();
            // HEAD: this plane's base values, loaded before this step's stores and copy
            // so that waiting for them waits for nothing younger
            float hbase[4] = {0.f, 0.f, 0.f, 0.f};
            if (HEAD && a.hbase && kb == 0 && yy < a.ny) {
#pragma unroll
                for (int t4 = 0; t4 < 4; ++t4) {
                    const int xx = x0 + 16 * t4 + m;
                    if (xx < a.nx) hbase[t4] = a.hbase[((int64_t)(z0 + p) * a.ny + yy) * a.nx + xx];
                }
            }
            flush();
            if (p + 2 <= n) copy_plane(z0 + p + 2, ring(k + 3));
            // The slot a lane reads is fixed per chunk except where the chunk's two taps
            // lie in different planes (taps 8 and 9): there both slots are read and each
            // lane keeps its own, so that every LDS read names one slot at compile time
            // (a read the compiler cannot place waits for the copy in flight).
            auto read_a = [&](int q, bf16x8(&A)[4]) {
                const int tap = 2 * q + (kb >> 1);
                const int dy = (tap / 3) % 3, dx = tap % 3;
                const int dz0 = (2 * q) / 9, dz1 = (2 * q + 1) / 9;
                const int base = (wave + dy) * kBX + m + dx;
#pragma unroll
                for (int t4 = 0; t4 < 4; ++t4) {
                    const int o = (base + 16 * t4) * kVS + chan;
                    uint4 av = *reinterpret_cast<const uint4 *>(&ring(k + dz0)[o]);
                    if (dz1 != dz0 && 2 * q + 1 < 27) {
                        // combined by masks: a select of the two loads would fold into
                        // one load from a selected slot
                        const uint4 a1 = *reinterpret_cast<const uint4 *>(&ring(k + dz1)[o]);
                        const uint32_t k1 = 0u - (uint32_t)(kb >> 1), k0 = ~k1;
                        av = make_uint4((av.x & k0) | (a1.x & k1), (av.y & k0) | (a1.y & k1), (av.z & k0) | (a1.z & k1),
                                        (av.w & k0) | (a1.w & k1));
                    }
                    if (tap >= 27) av = make_uint4(0u, 0u, 0u, 0u);
                    A[t4] = __builtin_bit_cast(bf16x8, av);
                }
            };
            f32x4 acc[4];
#pragma unroll
            for (int t4 = 0; t4 < 4; ++t4) acc[t4] = (f32x4){0.f, 0.f, 0.f, 0.f};
            bf16x8 Af[2][4];
            read_a(0, Af[0]);
#pragma unroll
            for (int q = 0; q < kKC; ++q) {
                if (q + 1 < kKC) read_a(q + 1, Af[(q + 1) & 1]);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int t4 = 0; t4 < 4; ++t4)
                    acc[t4] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(B[q], Af[q & 1][t4], acc[t4], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int t4 = 0; t4 < 4; ++t4) {
                float v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    v[i] = acc[t4][i] + bias[i];
                    if (a.relu) v[i] = fmaxf(v[i], 0.f);
                }
                const uint2 o = make_uint2((uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16),
                                           (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16));
                if (HEAD) {
                    // the head's sum in channel order, as unet_head_fwd forms it from the
                    // stored BF16 values: lanes of group kb add channels 4 kb .. 4 kb + 3
                    // and pass the sum to group kb + 1 (16 lanes up)
                    float hs = hb + hbase[t4];
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        if (g > 0) {
                            const float up = __shfl_up(hs, 16, 64);
                            if (kb == g) hs = up;
                        }
                        if (kb == g) {
                            hs = fmaf(hw[0], bf2f((uint16_t)(o.x & 0xffffu)), hs);
                            hs = fmaf(hw[1], bf2f((uint16_t)(o.x >> 16)), hs);
                            hs = fmaf(hw[2], bf2f((uint16_t)(o.y & 0xffffu)), hs);
                            hs = fmaf(hw[3], bf2f((uint16_t)(o.y >> 16)), hs);
                        }
                    }
                    if (t4 == 0) hpend0 = hs;
                    else if (t4 == 1) hpend1 = hs;
                    else if (t4 == 2) hpend2 = hs;
                    else hpend3 = hs;
                } else if (t4 == 0) pend0 = o;
                else if (t4 == 1) pend1 = o;
                else if (t4 == 2) pend2 = o;
                else pend3 = o;
                const int xx = x0 + 16 * t4 + m;
                if (a.y32 && yy < a.ny && xx < a.nx)
                    *reinterpret_cast<float4 *>(a.y32 + (((int64_t)p + z0) * a.ny + yy) * a.nx * a.cout +
                                                (int64_t)xx * a.cout + c) = make_float4(v[0], v[1], v[2], v[3]);
            }
            pend_z = z0 + p;
        }
    }
    flush();
}

// wt[ci][tap' * cout + co] = w[co][(26 - tap') * cin + ci]
__global__ void k_wtrans(const uint16_t *w, uint16_t *wt, int cin, int cout, int kpad_in, int kpad_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)cin * kpad_out) return;
    const int ci = (int)(i / kpad_out), kk = (int)(i % kpad_out);
    uint16_t v = 0;
    if (kk < 27 * cout) {
        const int tp = kk / cout, co = kk % cout;
        v = w[(int64_t)co * kpad_in + (26 - tp) * cin + ci];
    }
    wt[i] = v;
}

// ------------------------------------------------------------------ conv3d weight gradient
//
// dw[co][k] += sum_v dy[v][co] X(v, k) with X the im2col view of x: a GEMM whose
// reduction runs over the voxels.  On the 16x16x32 BF16 MFMA: M = output channel,
// N = k, K = 32 voxels per instruction.  A workgroup (4 waves) owns 16*NCO output
// channels x 128 k over a voxel range; per stage it stages 32 voxels of dy and of
// X into LDS transposed (voxels fastest), so each lane reads its 8-voxel fragment
// with one 16-byte LDS load; each wave accumulates NCO x 2 tiles of 16 x 16 in FP32
// and adds them to dw atomically at the end.
constexpr int kWgStage = 32;  // voxels per stage (the MFMA's K)
constexpr int kWgK = 128;     // k per workgroup
constexpr int kWgPad = 40;    // LDS row length (bf16): 32 voxels + 8 against bank conflicts

template <int NCO>
__global__ __launch_bounds__(256) void k_wgrad(const uint16_t *x, int ldx, int offx, const uint16_t *dy, int lddy,
                                               int offdy, int nz, int ny, int nx, int cin, int cout, int kpad,
                                               int64_t vper, float *dw, float *db) {
    __shared__ __attribute__((aligned(16))) uint16_t XT[kWgK][kWgPad];
    __shared__ __attribute__((aligned(16))) uint16_t DT[16 * NCO][kWgPad];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int k0 = blockIdx.x * kWgK, co0 = blockIdx.z * 16 * NCO;
    const int K = 27 * cin;
    const int64_t nvox = (int64_t)nz * ny * nx;
    const int64_t v0 = (int64_t)blockIdx.y * vper;
    const int64_t v1 = min(nvox, v0 + vper);
    // staging roles: X: voxel sv = tid / 8, two 8-wide k chunks c = tid % 8 and + 8
    const int sv = tid >> 3, sc = tid & 7;
    int ck[2], cdz[2], cdy[2], cdx[2], cci[2];
    bool cok[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int k = k0 + 8 * (sc + 8 * h);
        cok[h] = k < K;
        const int tap = cok[h] ? k / cin : 0;
        ck[h] = 8 * (sc + 8 * h);
        cci[h] = k - tap * cin;
        cdz[h] = tap / 9 - 1;
        cdy[h] = (tap / 3) % 3 - 1;
        cdx[h] = tap % 3 - 1;
    }
    // dy: voxel sv, channels 8 * sc .. when 8 * sc < 16 * NCO
    const bool dact = 8 * sc < 16 * NCO;
    f32x4 acc[NCO][2];
#pragma unroll
    for (int c = 0; c < NCO; ++c)
#pragma unroll
        for (int t = 0; t < 2; ++t) acc[c][t] = (f32x4){0.f, 0.f, 0.f, 0.f};
    float bacc = 0.f;
    const int m = lane & 15, q = lane >> 4;
    for (int64_t vs = v0; vs < v1; vs += kWgStage) {
        const int64_t v = vs + sv;
        const bool vok = v < v1;
        int xx = 0, yy = 0, zz = 0;
        if (vok) {
            xx = (int)(v % nx);
            const int64_t r = v / nx;
            yy = (int)(r % ny);
            zz = (int)(r / ny);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            uint4 val = make_uint4(0u, 0u, 0u, 0u);
            const int z2 = zz + cdz[h], y2 = yy + cdy[h], x2 = xx + cdx[h];
            if (vok && cok[h] && z2 >= 0 && z2 < nz && y2 >= 0 && y2 < ny && x2 >= 0 && x2 < nx) {
                const int64_t nb = ((int64_t)z2 * ny + y2) * nx + x2;
                val = *reinterpret_cast<const uint4 *>(x + nb * ldx + offx + cci[h]);
            }
            const uint16_t *e = reinterpret_cast<const uint16_t *>(&val);
#pragma unroll
            for (int i = 0; i < 8; ++i) XT[ck[h] + i][sv] = e[i];
        }
        if (dact) {
            uint4 val = make_uint4(0u, 0u, 0u, 0u);
            if (vok) val = *reinterpret_cast<const uint4 *>(dy + v * lddy + offdy + co0 + 8 * sc);
            const uint16_t *e = reinterpret_cast<const uint16_t *>(&val);
#pragma unroll
            for (int i = 0; i < 8; ++i) DT[8 * sc + i][sv] = e[i];
        }
        __syncthreads();
        bf16x8 A[NCO];
#pragma unroll
        for (int c = 0; c < NCO; ++c)
            A[c] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(&DT[16 * c + m][8 * q]));
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const bf16x8 B =
                __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(&XT[16 * (2 * wave + t) + m][8 * q]));
#pragma unroll
            for (int c = 0; c < NCO; ++c) acc[c][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[c], B, acc[c][t], 0, 0, 0);
        }
        if (db && blockIdx.x == 0 && tid < 16 * NCO)
            for (int i = 0; i < kWgStage; ++i) bacc += bf2f(DT[tid][i]);
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < NCO; ++c)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int k = k0 + 16 * (2 * wave + t) + m;
            if (k >= K) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = co0 + 16 * c + 4 * q + i;
                const float v = acc[c][t][i];
                if (v != 0.f) atomicAdd(&dw[(int64_t)co * kpad + k], v);
            }
        }
    if (db && blockIdx.x == 0 && tid < 16 * NCO) atomicAdd(&db[co0 + tid], bacc);
}

// ------------------------------------------------------------------ elementwise layers

__global__ void k_relu_bwd(const uint16_t *y, int ldy, int offy, uint16_t *d, int ldd, int offd, int64_t nvox, int c) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nvox * c) return;
    const int64_t v = i / c;
    const int ch = (int)(i % c);
    if (!(bf2f(y[v * ldy + offy + ch]) > 0.f)) d[v * ldd + offd + ch] = 0;
}

__global__ void k_pool_fwd(const uint16_t *x, int ldx, int offx, uint16_t *y, int ldy, int offy, int nz, int ny,
                           int nx, int c) {
    const int hz = nz / 2, hy = ny / 2, hx = nx / 2;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)hz * hy * hx * c) return;
    const int ch = (int)(i % c);
    const int64_t p = i / c;
    const int X = (int)(p % hx), Y = (int)((p / hx) % hy), Z = (int)(p / ((int64_t)hx * hy));
    float s = 0.f;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx)
                s += bf2f(x[(((int64_t)(2 * Z + dz) * ny + 2 * Y + dy) * nx + 2 * X + dx) * ldx + offx + ch]);
    y[p * ldy + offy + ch] = f2bf(0.125f * s);
}

__global__ void k_pool_bwd(const uint16_t *dy, int ldy, int offy, uint16_t *dx, int ldx, int offx, int nz, int ny,
                           int nx, int c) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nz * ny * nx * c) return;
    const int ch = (int)(i % c);
    const int64_t v = i / c;
    const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((int64_t)nx * ny));
    const int64_t p = ((int64_t)(z / 2) * (ny / 2) + y / 2) * (nx / 2) + x / 2;
    uint16_t *o = dx + v * ldx + offx + ch;
    *o = f2bf(bf2f(*o) + 0.125f * bf2f(dy[p * ldy + offy + ch]));
}

__global__ void k_up_fwd(const uint16_t *x, int ldx, int offx, uint16_t *y, int ldy, int offy, int nz, int ny, int nx,
                         int c) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nz * ny * nx * c) return;
    const int ch = (int)(i % c);
    const int64_t v = i / c;
    const int xx = (int)(v % nx), yy = (int)((v / nx) % ny), zz = (int)(v / ((int64_t)nx * ny));
    const int64_t p = ((int64_t)(zz / 2) * (ny / 2) + yy / 2) * (nx / 2) + xx / 2;
    y[v * ldy + offy + ch] = x[p * ldx + offx + ch];
}

__global__ void k_up_bwd(const uint16_t *dy, int ldy, int offy, uint16_t *dx, int ldx, int offx, int nz, int ny,
                         int nx, int c) {
    const int hz = nz / 2, hy = ny / 2, hx = nx / 2;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)hz * hy * hx * c) return;
    const int ch = (int)(i % c);
    const int64_t p = i / c;
    const int X = (int)(p % hx), Y = (int)((p / hx) % hy), Z = (int)(p / ((int64_t)hx * hy));
    float s = 0.f;
    for (int dz = 0; dz < 2; ++dz)
        for (int dyy = 0; dyy < 2; ++dyy)
            for (int ddx = 0; ddx < 2; ++ddx)
                s += bf2f(dy[(((int64_t)(2 * Z + dz) * ny + 2 * Y + dyy) * nx + 2 * X + ddx) * ldy + offy + ch]);
    dx[p * ldx + offx + ch] = f2bf(s);
}

// The same three layers on runs of 8 channels (16 bytes) per thread, for channel
// counts, row lengths and offsets that are multiples of 8 (every call the network
// makes); 32-bit index arithmetic (grids below 2^32 voxel-runs).
__device__ __forceinline__ void bf8_to_f(uint4 u, float (&f)[8]) {
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        f[2 * k] = __uint_as_float(w[k] << 16);
        f[2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
    }
}

__global__ void k_pool_fwd8(const uint16_t *x, int ldx, int offx, uint16_t *y, int ldy, int offy, uint32_t nz,
                            uint32_t ny, uint32_t nx, uint32_t c8) {
    const uint32_t hy = ny / 2, hx = nx / 2;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if ((uint64_t)i >= (uint64_t)(nz / 2) * hy * hx * c8) return;
    const uint32_t g = i % c8, p = i / c8;
    const uint32_t X = p % hx, Y = (p / hx) % hy, Z = p / (hx * hy);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        const uint64_t v = ((uint64_t)(2 * Z + (d >> 2)) * ny + 2 * Y + ((d >> 1) & 1)) * nx + 2 * X + (d & 1);
        float f[8];
        bf8_to_f(*reinterpret_cast<const uint4 *>(x + v * ldx + offx + 8 * g), f);
#pragma unroll
        for (int k = 0; k < 8; ++k) s[k] += f[k];
    }
    uint16_t o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = f2bf(0.125f * s[k]);
    *reinterpret_cast<uint4 *>(y + (uint64_t)p * ldy + offy + 8 * g) = *reinterpret_cast<const uint4 *>(o);
}

__global__ void k_up_fwd8(const uint16_t *x, int ldx, int offx, uint16_t *y, int ldy, int offy, uint32_t nz,
                          uint32_t ny, uint32_t nx, uint32_t c8) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if ((uint64_t)i >= (uint64_t)nz * ny * nx * c8) return;
    const uint32_t g = i % c8, v = i / c8;
    const uint32_t xx = v % nx, yy = (v / nx) % ny, zz = v / (nx * ny);
    const uint64_t p = ((uint64_t)(zz / 2) * (ny / 2) + yy / 2) * (nx / 2) + xx / 2;
    *reinterpret_cast<uint4 *>(y + (uint64_t)v * ldy + offy + 8 * g) =
        *reinterpret_cast<const uint4 *>(x + p * ldx + offx + 8 * g);
}

__global__ void k_head_fwd8(const uint16_t *x, int ldx, const float *w, const float *b, const float *base, float *out,
                            int64_t nvox, int c8) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvox) return;
    float s = b[0] + (base ? base[v] : 0.f);
    for (int g = 0; g < c8; ++g) {
        float f[8];
        bf8_to_f(*reinterpret_cast<const uint4 *>(x + v * ldx + 8 * g), f);
#pragma unroll
        for (int k = 0; k < 8; ++k) s = fmaf(w[8 * g + k], f[k], s);
    }
    out[v] = s;
}

__global__ void k_head_fwd(const uint16_t *x, int ldx, const float *w, const float *b, const float *base, float *out,
                           int64_t nvox, int c) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvox) return;
    float s = b[0] + (base ? base[v] : 0.f);
    for (int ch = 0; ch < c; ++ch) s = fmaf(w[ch], bf2f(x[v * ldx + ch]), s);
    out[v] = s;
}

__device__ __forceinline__ float block_sum(float v, float *red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    float t = 0.f;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
    __syncthreads();
    return t;
}

constexpr int kHeadMaxC = 32;  // channels of the 1x1x1 head (the first U-Net level)

// Grid-stride over the voxels with per-thread channel partials in registers, so
// each workgroup reduces and adds to dw / db once (not once per 256 voxels).
__global__ __launch_bounds__(256) void k_head_bwd(const uint16_t *x, int ldx, const float *w, const float *dout,
                                                  uint16_t *dx, float *dw, float *db, int64_t nvox, int c) {
    __shared__ float red[4];
    float part[kHeadMaxC];
#pragma unroll
    for (int ch = 0; ch < kHeadMaxC; ++ch) part[ch] = 0.f;
    float gsum = 0.f;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += (int64_t)gridDim.x * blockDim.x) {
        const float g = dout[v];
        gsum += g;
#pragma unroll
        for (int ch = 0; ch < kHeadMaxC; ++ch) {
            if (ch < c) {
                part[ch] += g * bf2f(x[v * ldx + ch]);
                dx[v * c + ch] = f2bf(g * w[ch]);
            }
        }
    }
#pragma unroll
    for (int ch = 0; ch < kHeadMaxC; ++ch) {
        if (ch < c) {
            const float s = block_sum(part[ch], red);
            if (threadIdx.x == 0) atomicAdd(&dw[ch], s);
        }
    }
    const float s = block_sum(gsum, red);
    if (threadIdx.x == 0) atomicAdd(db, s);
}

__global__ __launch_bounds__(256) void k_mse(const float *pred, const float *target, const uint8_t *mask,
                                             const float *weight, float *dout, float *loss, int64_t nvox,
                                             float inv_count) {
    __shared__ float red[4];
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float e = 0.f;
    if (v < nvox) {
        const float d = mask[v] ? pred[v] - target[v] : 0.f;
        const float wd = (weight ? weight[v] : 1.f) * d;
        dout[v] = 2.f * wd * inv_count;
        e = wd * d * inv_count;
    }
    const float s = block_sum(e, red);
    if (threadIdx.x == 0) atomicAdd(loss, s);
}

__global__ void k_adam(float *p, float *m, float *v, const float *g, uint16_t *pb, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    p[i] = pi;
    if (pb) pb[i] = f2bf(pi);
}

__global__ void k_to_bf16(const float *s, uint16_t *d, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = f2bf(s[i]);
}

__global__ void k_zero(uint32_t *d, int64_t nwords) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nwords) d[i] = 0u;
}

__global__ void k_features(const uint8_t *active, const uint8_t *ncat, const float *omega, float tau_ref,
                           uint16_t *feat, float *weight, float weight_power, float weight_cap, int nz, int ny,
                           int nx) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= (int64_t)nz * ny * nx) return;
    const int x = (int)(v % nx);
    // distances to the inlet and outlet faces in voxels, not fractions of the length,
    // so that a network trained on short domains transfers to longer ones
    const float xi = (float)x, xo = (float)(nx - 1 - x);
    float f[6] = {0.f, 0.f, 0.f, expf(-xi / 24.f), expf(-xi / 96.f), expf(-xo / 24.f)};
    float w = 0.f;
    if (active[v]) {
        f[0] = 1.f;
        const float tau = 1.f / omega[v];
        const float drel = fmaxf((tau - 0.5f) / (tau_ref - 0.5f), 1e-9f);
        f[1] = log10f(drel) / 3.f;
        f[2] = ncat ? (float)ncat[v] / 6.f : 0.f;
        w = fminf(weight_cap, powf(1.f / drel, weight_power));
    }
    uint16_t *o = feat + v * 16;
    for (int c = 0; c < 16; ++c) o[c] = c < 6 ? f2bf(f[c]) : (uint16_t)0;
    if (weight) weight[v] = w;
}

// y = ln(max(c, 0) + eps), or its inverse c = min(cmax, max(0, exp(y) - eps))
__global__ void k_log_map(const float *src, float *dst, int64_t n, float eps, int inverse, float cmax) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = src[i];
    dst[i] = inverse ? fminf(cmax, fmaxf(0.f, expf(v) - eps)) : logf(fmaxf(v, 0.f) + eps);
}

// start field of the solver from the network's log-space output: the prediction
// where the pore depth is at most depth_max, zero (the cold start) elsewhere
__global__ void k_start_field(const float *y, const uint8_t *depth, int depth_max, float eps, float cmax, float *c,
                              int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    c[i] = (int)depth[i] <= depth_max ? fminf(cmax, fmaxf(0.f, expf(y[i]) - eps)) : 0.f;
}

// corrector of the effective-diffusivity problem: the field minus the linear profile
// between the two Dirichlet faces, in units of the mean gradient (or its inverse)
__global__ void k_corrector(const float *src, float *dst, int64_t n, int nx, float c_in, float c_out, int inverse,
                            float cmax) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = (float)(i % nx);
    const float lin = c_in + (c_out - c_in) * (x + 0.5f) / (float)nx;
    const float scale = (float)nx / (c_in - c_out);
    dst[i] = inverse ? fminf(cmax, fmaxf(0.f, lin + src[i] / scale)) : (src[i] - lin) * scale;
}

// D = A B (16x32 by 32x16) through the conv kernel's fragment mapping
__global__ void k_mfma_selftest(const float *a, const float *b, float *d) {
    const int lane = threadIdx.x;
    const int m = lane & 15, kb = lane >> 4;
    uint16_t av[8], bv[8];
    for (int j = 0; j < 8; ++j) {
        av[j] = f2bf(a[m * 32 + 8 * kb + j]);
        bv[j] = f2bf(b[(8 * kb + j) * 16 + m]);
    }
    const bf16x8 A = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(av));
    const bf16x8 B = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(bv));
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, acc, 0, 0, 0);
    for (int i = 0; i < 4; ++i) d[(4 * kb + i) * 16 + m] = acc[i];
}

dim3 grid1(int64_t n, int bs = 256) { return dim3((unsigned)((n + bs - 1) / bs)); }

bool ch_ok(int ld, int off, int c) { return ld > 0 && off >= 0 && c > 0 && off + c <= ld; }

// channel count, row lengths and offsets all in runs of 8 (16-byte loads and stores)
bool runs8(int c, int ld1, int off1, int ld2, int off2) { return ((c | ld1 | off1 | ld2 | off2) & 7) == 0; }

}  // namespace

extern "C" {

int32_t unet_kpad(int32_t cin) { return kpad_of(cin); }

// both convolution entry points: a.x2 is a.x and a.cin1 a.cin for a single input
static int launch_conv(ConvArgs a, int64_t nx2, int64_t ny2, int64_t nz2, void *stream) {
    const int nx = a.nx, ny = a.ny, nz = a.nz, cin = a.cin, cout = a.cout;
    if (!a.x || !a.x2 || !a.w || (!a.y && !a.hout) || nz <= 0 || ny <= 0 || nx <= 0 || cin % 16 || a.cin1 % 16 ||
        a.cin1 <= 0 || a.cin1 > cin || !ch_ok(a.ldx, a.offx, a.cin1) || (a.cin1 < cin && !ch_ok(a.ldx2, a.offx2, cin - a.cin1)) ||
        !ch_ok(a.ldy, a.offy, cout) || (a.ldx % 8) || (a.offx % 8) || (a.ldx2 % 8) || (a.offx2 % 8) || (a.ldy % 8) ||
        (a.offy % 8))
        return -1;
    if (cout % 16 || nz > 65535) return -1;
    if ((reinterpret_cast<uintptr_t>(a.x) | reinterpret_cast<uintptr_t>(a.x2) | reinterpret_cast<uintptr_t>(a.w) |
         reinterpret_cast<uintptr_t>(a.y) | reinterpret_cast<uintptr_t>(a.y32)) & 15)
        return -1;  // 16-byte vector loads and stores
    const int tiles = cout / 16;
    const int nt = 1;  // one 16-channel tile per wave: its 14 weight fragments stay in registers
    const int64_t plane_bytes = 2 * (int64_t)ny * nx * a.ldx, xbytes = plane_bytes * nz;
    const int64_t plane2_bytes = 2 * ny2 * nx2 * a.ldx2, x2bytes = plane2_bytes * nz2;
    const int64_t wbytes = 2 * (int64_t)cout * kpad_of(cin);
    if (xbytes > kMaxX || x2bytes > kMaxX || wbytes > kMaxX) return -1;
    a.kpad = kpad_of(cin);
    a.xbytes = (uint32_t)xbytes;
    a.plane_bytes = (uint32_t)plane_bytes;
    a.x2bytes = (uint32_t)x2bytes;
    a.plane2_bytes = (uint32_t)plane2_bytes;
    a.wbytes = (uint32_t)wbytes;
    const int64_t nxy = (int64_t)((nx + kTX - 1) / kTX) * ((ny + kTY - 1) / kTY);
    if (nxy > 0x7fffffff) return -1;
    if (cin == kCC && a.cin1 == cin) {
        // one stage: the z-marching form, runs of zr planes (4 .. 32), about three
        // rounds of two workgroups per CU on a large grid (timed best among 768 ..
        // 6144 workgroups)
        const int64_t zr = std::min<int64_t>(32, std::max<int64_t>(4, nxy * (tiles / nt) * nz / kZmWorkgroups));
        const dim3 g((unsigned)nxy, (unsigned)((nz + zr - 1) / zr), (unsigned)(tiles / nt)), blk(256);
        (void)hipGetLastError();
        if (a.hout)
            hipLaunchKernelGGL(k_conv_zm<true>, g, blk, 0, static_cast<hipStream_t>(stream), a, (int)zr);
        else
            hipLaunchKernelGGL(k_conv_zm<false>, g, blk, 0, static_cast<hipStream_t>(stream), a, (int)zr);
        return status(hipGetLastError());
    }
    const bool large = nxy * ((nz + 3) / 4) * (tiles / nt) >= kZcLargeGrid;
    const int zc = large ? 4 : 3;
    const dim3 g((unsigned)nxy, (unsigned)((nz + zc - 1) / zc), (unsigned)(tiles / nt)), blk(256);
    hipStream_t st = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    if (large)
        hipLaunchKernelGGL((k_conv_fwd<1, 4>), g, blk, 0, st, a);
    else
        hipLaunchKernelGGL((k_conv_fwd<1, 3>), g, blk, 0, st, a);
    return status(hipGetLastError());
}

int unet_conv3d_fwd(const uint16_t *x, int32_t ldx, int32_t offx, const uint16_t *w, const float *b, uint16_t *y,
                    int32_t ldy, int32_t offy, float *y32, int32_t nz, int32_t ny, int32_t nx, int32_t cin,
                    int32_t cout, int32_t relu, void *stream) {
    ConvArgs a{x, w, b, y, y32, ldx, offx, ldy, offy, nz, ny, nx, cin, cout, 0, relu, 0, 0, 0,
               x, ldx, offx, cin, 0, 0, 0, nullptr, nullptr, nullptr, nullptr};
    return launch_conv(a, nx, ny, nz, stream);
}

int unet_conv3d_fwd_head(const uint16_t *x, int32_t ldx, int32_t offx, const uint16_t *w, const float *b,
                         const float *hw, const float *hb, const float *base, float *out, int32_t nz, int32_t ny,
                         int32_t nx, void *stream) {
    if (!hw || !hb || !out) return -1;
    // 16 -> 16 channels with ReLU, then the head; the BF16 outputs are not stored
    ConvArgs a{x, w, b, nullptr, nullptr, ldx, offx, 16, 0, nz, ny, nx, 16, 16, 0, 1, 0, 0, 0,
               x, ldx, offx, 16, 0, 0, 0, hw, hb, base, out};
    return launch_conv(a, nx, ny, nz, stream);
}

int unet_conv3d_fwd_cat(const uint16_t *x, int32_t ldx, int32_t offx, int32_t cin1, const uint16_t *x2, int32_t ldx2,
                        int32_t offx2, const uint16_t *w, const float *b, uint16_t *y, int32_t ldy, int32_t offy,
                        float *y32, int32_t nz, int32_t ny, int32_t nx, int32_t cin, int32_t cout, int32_t relu,
                        void *stream) {
    if (nz % 2 || ny % 2 || nx % 2) return -1;  // x2 holds the half-resolution grid
    ConvArgs a{x, w, b, y, y32, ldx, offx, ldy, offy, nz, ny, nx, cin, cout, 0, relu, 0, 0, 0,
               x2, ldx2, offx2, cin1, 1, 0, 0, nullptr, nullptr, nullptr, nullptr};
    if (cin1 >= cin) return -1;
    return launch_conv(a, nx / 2, ny / 2, nz / 2, stream);
}

int unet_conv3d_wtrans(const uint16_t *w, uint16_t *wt, int32_t cin, int32_t cout, void *stream) {
    if (!w || !wt || cin <= 0 || cout <= 0) return -1;
    const int64_t n = (int64_t)cin * kpad_of(cout);
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_wtrans, grid1(n), dim3(256), 0, static_cast<hipStream_t>(stream), w, wt, cin, cout,
                       kpad_of(cin), kpad_of(cout));
    return status(hipGetLastError());
}

int unet_conv3d_wgrad(const uint16_t *x, int32_t ldx, int32_t offx, const uint16_t *dy, int32_t lddy, int32_t offdy,
                      int32_t nz, int32_t ny, int32_t nx, int32_t cin, int32_t cout, float *dw, float *db,
                      void *stream) {
    if (!x || !dy || !dw || nz <= 0 || ny <= 0 || nx <= 0 || !ch_ok(ldx, offx, cin) || !ch_ok(lddy, offdy, cout))
        return -1;
    if (cin % 16 || cout % 16 || ldx % 8 || offx % 8 || lddy % 8 || offdy % 8) return -1;
    const int64_t nvox = (int64_t)nz * ny * nx;
    const int nco = cout % 64 == 0 ? 4 : (cout % 32 == 0 ? 2 : 1);
    // enough workgroups to fill the device: the voxel range per workgroup shrinks
    // for layers with few (k, channel) tiles
    const int64_t tiles = (int64_t)((27 * cin + kWgK - 1) / kWgK) * (cout / (16 * nco));
    int64_t vper = 4096;
    while (vper > 512 && tiles * ((nvox + vper - 1) / vper) < 2048) vper >>= 1;
    const dim3 g((unsigned)((27 * cin + kWgK - 1) / kWgK), (unsigned)((nvox + vper - 1) / vper),
                 (unsigned)(cout / (16 * nco)));
    (void)hipGetLastError();
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const int kp = kpad_of(cin);
    switch (nco) {
        case 4: hipLaunchKernelGGL(k_wgrad<4>, g, dim3(256), 0, st, x, ldx, offx, dy, lddy, offdy, nz, ny, nx, cin, cout, kp, vper, dw, db); break;
        case 2: hipLaunchKernelGGL(k_wgrad<2>, g, dim3(256), 0, st, x, ldx, offx, dy, lddy, offdy, nz, ny, nx, cin, cout, kp, vper, dw, db); break;
        default: hipLaunchKernelGGL(k_wgrad<1>, g, dim3(256), 0, st, x, ldx, offx, dy, lddy, offdy, nz, ny, nx, cin, cout, kp, vper, dw, db); break;
    }
    return status(hipGetLastError());
}

int unet_relu_bwd(const uint16_t *y, int32_t ldy, int32_t offy, uint16_t *dy, int32_t ldd, int32_t offd, int64_t nvox,
                  int32_t c, void *stream) {
    if (!y || !dy || !ch_ok(ldy, offy, c) || !ch_ok(ldd, offd, c) || nvox <= 0) return -1;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_relu_bwd, grid1(nvox * c), dim3(256), 0, static_cast<hipStream_t>(stream), y, ldy, offy, dy,
                       ldd, offd, nvox, c);
    return status(hipGetLastError());
}

int unet_pool_fwd(const uint16_t *x, int32_t ldx, int32_t offx, uint16_t *y, int32_t ldy, int32_t offy, int32_t nz,
                  int32_t ny, int32_t nx, int32_t c, void *stream) {
    if (!x || !y || (nz | ny | nx) & 1 || nz <= 0 || !ch_ok(ldx, offx, c) || !ch_ok(ldy, offy, c)) return -1;
    (void)hipGetLastError();
    if (runs8(c, ldx, offx, ldy, offy) && (int64_t)nz * ny * nx / 8 * (c / 8) < ((int64_t)1 << 32))
        hipLaunchKernelGGL(k_pool_fwd8, grid1((int64_t)nz * ny * nx / 8 * (c / 8)), dim3(256), 0,
                           static_cast<hipStream_t>(stream), x, ldx, offx, y, ldy, offy, (uint32_t)nz, (uint32_t)ny,
                           (uint32_t)nx, (uint32_t)(c / 8));
    else
        hipLaunchKernelGGL(k_pool_fwd, grid1((int64_t)nz * ny * nx / 8 * c), dim3(256), 0,
                           static_cast<hipStream_t>(stream), x, ldx, offx, y, ldy, offy, nz, ny, nx, c);
    return status(hipGetLastError());
}

int unet_pool_bwd(const uint16_t *dy, int32_t ldy, int32_t offy, uint16_t *dx, int32_t ldx, int32_t offx, int32_t nz,
                  int32_t ny, int32_t nx, int32_t c, void *stream) {
    if (!dy || !dx || (nz | ny | nx) & 1 || nz <= 0 || !ch_ok(ldx, offx, c) || !ch_ok(ldy, offy, c)) return -1;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_pool_bwd, grid1((int64_t)nz * ny * nx * c), dim3(256), 0, static_cast<hipStream_t>(stream),
                       dy, ldy, offy, dx, ldx, offx, nz, ny, nx, c);
    return status(hipGetLastError());
}

int unet_up_fwd(const uint16_t *x, int32_t ldx, int32_t offx, uint16_t *y, int32_t ldy, int32_t offy, int32_t nz,
                int32_t ny, int32_t nx, int32_t c, void *stream) {
    if (!x || !y || (nz | ny | nx) & 1 || nz <= 0 || !ch_ok(ldx, offx, c) || !ch_ok(ldy, offy, c)) return -1;
    (void)hipGetLastError();
    if (runs8(c, ldx, offx, ldy, offy) && (int64_t)nz * ny * nx * (c / 8) < ((int64_t)1 << 32))
        hipLaunchKernelGGL(k_up_fwd8, grid1((int64_t)nz * ny * nx * (c / 8)), dim3(256), 0,
                           static_cast<hipStream_t>(stream), x, ldx, offx, y, ldy, offy, (uint32_t)nz, (uint32_t)ny,
                           (uint32_t)nx, (uint32_t)(c / 8));
    else
        hipLaunchKernelGGL(k_up_fwd, grid1((int64_t)nz * ny * nx * c), dim3(256), 0, static_cast<hipStream_t>(stream),
                           x, ldx, offx, y, ldy, offy, nz, ny, nx, c);
    return status(hipGetLastError());
}

int unet_up_bwd(const uint16_t *dy, int32_t ldy, int32_t offy, uint16_t *dx, int32_t ldx, int32_t offx, int32_t nz,
                int32_t ny, int32_t nx, int32_t c, void *stream) {
    if (!dy || !dx || (nz | ny | nx) & 1 || nz <= 0 || !ch_ok(ldx, offx, c) || !ch_ok(ldy, offy, c)) return -1;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_up_bwd, grid1((int64_t)nz * ny * nx / 8 * c), dim3(256), 0,
                       static_cast<hipStream_t>(stream), dy, ldy, offy, dx, ldx, offx, nz, ny, nx, c);
    return status(hipGetLastError());
}

int unet_head_fwd(const uint16_t *x, int32_t ldx, const float *w, const float *b, const float *base, float *out,
                  int64_t nvox, int32_t c, void *stream) {
    if (!x || !w || !b || !out || nvox <= 0 || c <= 0 || ldx < c) return -1;
    (void)hipGetLastError();
    if (runs8(c, ldx, 0, 8, 0))
        hipLaunchKernelGGL(k_head_fwd8, grid1(nvox), dim3(256), 0, static_cast<hipStream_t>(stream), x, ldx, w, b,
                           base, out, nvox, c / 8);
    else
        hipLaunchKernelGGL(k_head_fwd, grid1(nvox), dim3(256), 0, static_cast<hipStream_t>(stream), x, ldx, w, b, base,
                           out, nvox, c);
    return status(hipGetLastError());
}

int unet_head_bwd(const uint16_t *x, int32_t ldx, const float *w, const float *dout, uint16_t *dx, float *dw,
                  float *db, int64_t nvox, int32_t c, void *stream) {
    if (!x || !w || !dout || !dx || !dw || !db || nvox <= 0 || c <= 0 || c > kHeadMaxC || ldx < c) return -1;
    (void)hipGetLastError();
    const dim3 g((unsigned)std::min<int64_t>((nvox + 255) / 256, 1024));
    hipLaunchKernelGGL(k_head_bwd, g, dim3(256), 0, static_cast<hipStream_t>(stream), x, ldx, w, dout, dx, dw, db,
                       nvox, c);
    return status(hipGetLastError());
}

int unet_mse(const float *pred, const float *target, const uint8_t *mask, const float *weight, float *dout,
             float *loss, int64_t nvox, int64_t count, void *stream) {
    if (!pred || !target || !mask || !dout || !loss || nvox <= 0 || count <= 0) return -1;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_mse, grid1(nvox), dim3(256), 0, static_cast<hipStream_t>(stream), pred, target, mask, weight,
                       dout, loss, nvox, 1.0f / (float)count);
    return status(hipGetLastError());
}

int unet_adam(float *p, float *m, float *v, const float *g, uint16_t *pb, int64_t n, float lr, float beta1,
              float beta2, float eps, int32_t t, void *stream) {
    if (!p || !m || !v || !g || n <= 0 || t < 1) return -1;
    const float c1 = 1.f / (1.f - powf(beta1, (float)t)), c2 = 1.f / (1.f - powf(beta2, (float)t));
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_adam, grid1(n), dim3(256), 0, static_cast<hipStream_t>(stream), p, m, v, g, pb, n, lr, beta1,
                       beta2, eps, c1, c2);
    return status(hipGetLastError());
}

int unet_to_bf16(const float *src, uint16_t *dst, int64_t n, void *stream) {
    if (!src || !dst || n <= 0) return -1;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_to_bf16, grid1(n), dim3(256), 0, static_cast<hipStream_t>(stream), src, dst, n);
    return status(hipGetLastError());
}

int unet_zero(void *dst, int64_t bytes, void *stream) {
    if (!dst || bytes < 0 || (bytes & 3)) return -1;
    if (bytes == 0) return 0;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_zero, grid1(bytes / 4), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<uint32_t *>(dst), bytes / 4);
    return status(hipGetLastError());
}

int unet_features(const uint8_t *active, const uint8_t *n_cat, const float *omega, float tau_ref, uint16_t *feat,
                  float *weight, float weight_power, float weight_cap, int32_t nz, int32_t ny, int32_t nx,
                  void *stream) {
    if (!active || !omega || !feat || nz <= 0 || ny <= 0 || nx <= 0 || !(tau_ref > 0.5f)) return -1;
    if (weight && !(weight_cap >= 1.f && weight_power >= 0.f && weight_power <= 4.f)) return -1;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_features, grid1((int64_t)nz * ny * nx), dim3(256), 0, static_cast<hipStream_t>(stream),
                       active, n_cat, omega, tau_ref, feat, weight, weight_power, weight_cap, nz, ny, nx);
    return status(hipGetLastError());
}

int unet_log_map(const float *src, float *dst, int64_t n, float eps, int32_t inverse, float cmax, void *stream) {
    if (!src || !dst || n <= 0 || !(eps > 0.f) || !(cmax > 0.f)) return -1;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_log_map, grid1(n), dim3(256), 0, static_cast<hipStream_t>(stream), src, dst, n, eps,
                       inverse ? 1 : 0, cmax);
    return status(hipGetLastError());
}

int unet_start_field(const float *y, const uint8_t *depth, int32_t depth_max, float eps, float cmax, float *c,
                     int64_t n, void *stream) {
    if (!y || !depth || !c || n <= 0 || depth_max < 0 || !(eps > 0.f) || !(cmax > 0.f)) return -1;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_start_field, grid1(n), dim3(256), 0, static_cast<hipStream_t>(stream), y, depth, depth_max,
                       eps, cmax, c, n);
    return status(hipGetLastError());
}

int unet_corrector_map(const float *src, float *dst, int64_t nvox, int32_t nx, float c_in, float c_out,
                       int32_t inverse, float cmax, void *stream) {
    if (!src || !dst || nvox <= 0 || nx <= 0 || nvox % nx || !(c_in != c_out) || !(cmax > 0.f)) return -1;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_corrector, grid1(nvox), dim3(256), 0, static_cast<hipStream_t>(stream), src, dst, nvox, nx,
                       c_in, c_out, inverse ? 1 : 0, cmax);
    return status(hipGetLastError());
}

int unet_mfma_selftest(const float *a, const float *b, float *d, void *stream) {
    if (!a || !b || !d) return -1;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_mfma_selftest, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), a, b, d);
    return status(hipGetLastError());
}

}  // extern "C"
