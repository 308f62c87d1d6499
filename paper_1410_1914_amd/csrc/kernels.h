// Device data structures and launch entry points of the D3Q7 kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cl {

// Per-instance constants, device resident (one entry per structure of a batch).
struct alignas(64) InstDev {
    int32_t nx, ny, nz, nsx;  // simulated grid, segments per row
    int64_t seg_base;         // first global segment of the instance
    int64_t nseg;             // segments of the instance
    // Stored populations are g_i = f_i - w_i c_sh(x) with c_sh(x) = sh0 - slope * x
    // (the linear empty-box profile for Dirichlet problems, a constant when reacting).
    double sh0, slope;
    double pull_dx;           // w1 * slope: added to a population pulled from x - 1
    double abb_in;            // 2 w1 (c_in - c_sh(0)): anti-bounce-back at x = 0
    double abb_out;           // 2 w1 (c_out - c_sh(nx - 1)): anti-bounce-back at x = nx
    double k;                 // first-order rate per catalyst face
    double w0, w1;            // rest and moving weights
    float om_pore, om_ion;    // relaxation rates when not stored per voxel
};

// Everything a wave needs to update one segment, a window of up to 64 voxels
// consecutive in grid order (one bit per lane; see Prepared for the two ways the
// grid is cut into windows).  Built once on the host; the stream-collide kernel
// reads it with a few scalar loads instead of recomputing neighbour rows and bit
// shifts per step.  Lane l lies at x = x0 + l, or at x = l - brk on the next row
// for l >= brk.
struct SegRec {
    uint64_t m;              // lanes that are simulated (fluid)
    uint64_t left, right;    // lanes whose x-1 / x+1 neighbour is fluid (x faces excluded)
    uint64_t nb[4];          // fluid masks of the lanes' neighbours in y-1, y+1, z-1, z+1
    uint64_t ion;            // ionomer lanes (relaxation rate from the phase)
    uint64_t n0, n1, n2;     // bit planes of n, the catalyst face-neighbour count, of reacting lanes
    uint32_t pre;            // global compact index of the first fluid lane
    uint32_t pnb[4];         // the same for the four neighbour windows
    uint32_t v0;             // grid index (within the instance) of lane 0
    uint16_t x0;             // x of lane 0
    uint8_t brk;             // first lane on the next row (64: none)
    uint8_t len;             // lanes inside the grid
    uint16_t inst, pad;      // instance
};
static_assert(sizeof(SegRec) == 120, "SegRec layout");

// Quantities reduced per instance, in this order.
enum { Q_JIN = 0, Q_JOUT, Q_JINT, Q_RATE, Q_MASS, Q_DCMAX, Q_CMAX, Q_BAD, NQ };

struct Lattice {
    const SegRec *rec;        // per segment of every instance
    const float *omega;       // per fluid voxel 1/tau (Knudsen problems), else null
    const InstDev *inst;
    uint32_t stride;          // fluid voxels rounded up to 64; a lattice is 7 * stride floats in blocks of
                              // 7 x 64 (one block per 64 compact voxels), 7 * stride * 4 < 2^32
};

struct StepLaunch {
    int32_t waves;            // waves per workgroup: 1, 2, 4, 8
    int32_t spw;              // segments per wave: 1, 2, 4
    int32_t xcd;              // XCD-aware block order
    int32_t nblk;             // workgroups
    int32_t nent;             // entries of the list
    const uint32_t *list;     // segments with fluid of the live instances, in grid order
    const uint32_t *list_inst;// instance of each list entry (several instances), so a wave can load
                              // its instance constants in parallel with its segment record
    int32_t single;           // 1: one instance (its constants load without waiting for the record)
    int32_t reverse;          // 1: walk each XCD's part of the list from its end (alternate steps, so each
                              // step starts on the segments the previous one touched last, still cached)
};

// Two time steps per launch (one instance).  A workgroup owns one 64-voxel x range
// (segment column s) and `by` consecutive rows in y, and marches through `zc`
// consecutive planes in z: the first step of each plane (tile rows, the two rows
// beside the tile in y, the voxel before and after the x range) lands in LDS, the
// second step reads it there and writes the lattice.
struct Step2Launch {
    int32_t by;               // rows per tile: 4, 6 or 8
    int32_t zc;               // planes per chunk
    int32_t nty, ncz;         // tiles in y, chunks in z
    int32_t nblk;             // nsx * nty * ncz workgroups
    int32_t xcd;              // XCD-aware block order
};

struct MeasureLaunch {
    int32_t nblk;
    const int4 *blk;          // per workgroup: {instance, block within instance, blocks of instance, partial slot}
    double *partial;          // [nblk][NQ]
    int32_t update_snap;
    float *csnap;             // per fluid voxel concentration snapshot
};

hipError_t launch_step(const Lattice &L, const StepLaunch &S, bool knudsen, bool react, const float *fin,
                       float *fout, hipStream_t st);
// Two steps from fin to fout (instance 0 of L only).
hipError_t launch_step2(const Lattice &L, const Step2Launch &S, bool knudsen, bool react, const float *fin,
                        float *fout, hipStream_t st);
hipError_t launch_measure(const Lattice &L, const MeasureLaunch &M, bool react, const float *f, hipStream_t st);
// results[i*NQ + q] from partials of blocks [base_i, base_i + count_i): ranges[i] = {base, count}
hipError_t launch_finish(const double *partial, const int2 *ranges, int32_t ninst, double *results, hipStream_t st);

// Dense <-> compact conversions over every segment of the instances in blk
// (entries {instance, first local segment}, four segments per 256-thread block).
hipError_t launch_init_eq(const Lattice &L, int32_t nblk, const int2 *blk, bool react, const float *c_dense,
                          const int64_t *dense_base, float *f, float *csnap, hipStream_t st);
hipError_t launch_set_pop(const Lattice &L, int32_t nblk, const int2 *blk, const float *f_dense,
                          const int64_t *dense_base, int64_t dense_stride, float *f, hipStream_t st);
hipError_t launch_get_pop(const Lattice &L, int32_t nblk, const int2 *blk, const float *f,
                          const int64_t *dense_base, int64_t dense_stride, float *f_dense, hipStream_t st);
hipError_t launch_conc(const Lattice &L, int32_t nblk, const int2 *blk, bool react, const float *f,
                       const int64_t *dense_base, float *c_dense, hipStream_t st);

// LBM_OK, or LBM_ERR_HIP with the failing call kept for lbm_last_error.
int record_error(hipError_t e, const char *where);

}  // namespace cl
