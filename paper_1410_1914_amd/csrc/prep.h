// Host-side preprocessing of a catalyst-layer structure into the per-segment
// bitmasks and compact per-fluid-voxel arrays the stream-collide kernels read.
#pragma once

#include <cstdint>
#include <mutex>
#include <vector>

#include "../../include/lbm.h"

namespace cl {

constexpr int kSeg = 64;  // voxels per row segment = one wave64, one 64-bit mask word

struct Prepared {
    lbm_params params{};
    int mode = 0;
    bool knudsen = false;
    int nx = 0, ny = 0, nz = 0;  // simulated grid
    int nx_struct = 0;
    int nsx = 0;                 // segments per row
    int64_t nseg = 0;
    int64_t n_fluid = 0;
    bool percolates = false;
    double d0 = 0, d_ref = 0, d0_lat = 0;
    double sh0 = 0, slope = 0;   // stored populations are shifted by w_i (sh0 - slope * x)
    double w0 = 0.25, w1 = 0.125;
    float om_pore = 1.f, om_ion = 1.f;  // relaxation rates when not per voxel
    // dense over the simulated grid
    std::vector<uint8_t> phase;  // phase ids, the reservoir plane included
    std::vector<uint8_t> active, n_cat;
    std::vector<float> omega_dense;
    // Segments: windows of up to 64 voxels consecutive in x-fastest (grid) order,
    // one wave each.  Row layout: every row starts a window (nsx windows per row,
    // the last one short when nx is not a multiple of 64).  Flat layout (rows of
    // 64 k + 1 voxels, i.e. the reservoir plane's 257): windows run on across row
    // ends, restarting only at each plane and at rows 1 and ny - 1, so a window
    // spans at most two rows and its y and z neighbours lie at one flat offset
    // for all its lanes; no one-voxel segment is left at the end of each row.
    bool flat = false;
    std::vector<uint32_t> win_v0;  // grid index of lane 0
    std::vector<uint8_t> win_len;  // lanes inside the grid
    std::vector<uint64_t> m_fluid, m_ion, m_react, m_cat;
    std::vector<uint32_t> prefix;  // compact index of the first fluid voxel of the segment
    // compact (fluid voxels in x-fastest order)
    std::vector<float> omega_c;
};

// Device assistance for prepare(): the 13-direction pore size and the reach from
// the Dirichlet faces run on the device (lbm_pore_size_device, lbm_reach_device)
// in a caller-owned scratch buffer, on `stream`.  The results are identical to the
// host computation.  `mu` serialises the device sections of concurrent calls that
// share the scratch.
struct DeviceAssist {
    void *scratch = nullptr;
    size_t bytes = 0;
    void *stream = nullptr;
    std::mutex *mu = nullptr;
};

// Scratch bytes prepare() needs with device assistance for a structure of g.
size_t prep_scratch_bytes(const lbm_grid &g, const lbm_params &p);

// Returns an LBM_* status.  dev: optional device assistance (may be null).
int prepare(const lbm_grid &g, const uint8_t *phase, const lbm_params &p, Prepared &out,
            const DeviceAssist *dev = nullptr);

// Distance (6-neighbour steps through active voxels, periodic in y and z) of every
// simulated voxel from the pore voxels joined to a Dirichlet face through pore
// voxels alone: 0 on those pores, 1..254 beyond them, 255 for inactive voxels, for
// voxels farther than 254 steps and for voxels no such path reaches.
void pore_depth(const Prepared &p, uint8_t *depth);

// 13-direction averaged pore size (voxel edges) of every voxel of `pore`.
void pore_size_13(int nx, int ny, int nz, const uint8_t *pore, std::vector<double> &dp);

}  // namespace cl
