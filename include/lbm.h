/*
 * lbm.h — C ABI of the MI355X (gfx950) D3Q7 reactive-diffusion lattice Boltzmann
 * solver for voxelised catalyst-layer structures.
 *
 * Method: Chen, Wu, Kang, Holby, Tao, "Nanoscale study of reactive transport in
 * catalyst layer of proton exchange membrane fuel cells with precious and
 * non-precious catalysts using lattice Boltzmann method", arXiv 1410.1914.
 *   - phases and local diffusivity: Section 3.1 (Eqs. 7-9), Section 3.2 (Eqs. 14-15);
 *   - pore size for Knudsen diffusion: 13-direction averaging, Section 2.1.3;
 *   - proton conduction: Section 3.3 (Eq. 16);
 *   - first-order surface reaction: Section 3.4 (Eqs. 17b, 18a) with uniform
 *     ionomer potential (Section 3.5.2);
 *   - boundary conditions: Section 3.5.1 (Eq. 19) and 3.5.2 (Eqs. 20a, 20b);
 *   - LBM evolution, equilibrium, moments and tau-D relation: Section 4,
 *     Eqs. (21)-(24), on the D3Q7 lattice (rest weight w0, c_s^2 = (1 - w0)/3).
 *
 * Conventions
 *   - Every function returns an int status: LBM_OK (0), LBM_NOT_CONVERGED (1,
 *     results readable but flagged), or a negative error.  No exception, abort or
 *     exit crosses this boundary.
 *   - Arrays named *_host are host memory; arrays named *_dev are device memory
 *     on the device current when lbm_bind was called.
 *   - Dense voxel arrays are x fastest: v = (z*ny + y)*nx + x.  Population arrays
 *     are [7][N] in the order rest, +x, -x, +y, -y, +z, -z.
 *   - Lattice units: dx = dt = 1.  All scalars are FP64 at the ABI; distributions
 *     are FP32 on the device, reductions FP64.
 *   - Ownership: the caller owns every pointer it passes.  The phase map is copied
 *     by lbm_create.  The device workspace handed to lbm_bind must stay allocated
 *     until lbm_destroy (or a re-bind).  The library allocates no device memory.
 *   - Streams: all device work is enqueued on the stream given to lbm_bind.
 *     Functions that return host values synchronise that stream.
 *   - Threading: a solver handle must not be used by two threads at once.
 */
#ifndef PAPER_1410_1914_AMD_LBM_H
#define PAPER_1410_1914_AMD_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 1

/* phase ids of the input map (Section 2: pore, carbon, Pt, ionomer) */
enum { LBM_PORE = 0, LBM_CARBON = 1, LBM_PT = 2, LBM_IONOMER = 3 };

/* problems (Section 3.5): effective O2 diffusivity, reactive O2 transport,
 * effective proton conductivity (ionomer is the only conducting phase) */
enum { LBM_MODE_DEFF = 0, LBM_MODE_REACT = 1, LBM_MODE_PROTON = 2 };

enum {
    LBM_OK = 0,
    LBM_NOT_CONVERGED = 1,
    LBM_ERR_INVALID_ARG = -1,   /* NULL pointer, bad size or parameter        */
    LBM_ERR_BAD_PHASE = -2,     /* phase id outside 0..3                       */
    LBM_ERR_WRONG_MODE = -3,    /* e.g. lbm_deff on a reactive problem         */
    LBM_ERR_NO_PERCOLATION = -4,/* no transport path between the Dirichlet faces
                                   (lbm_deff still returns 0 through its output) */
    LBM_ERR_DIVERGED = -5,      /* NaN or Inf in the distributions             */
    LBM_ERR_HIP = -6,           /* a HIP runtime call failed                   */
    LBM_ERR_UNBOUND = -7,       /* no workspace bound yet                      */
    LBM_ERR_WORKSPACE = -8,     /* workspace too small or misaligned           */
    LBM_ERR_UNSTABLE = -9       /* k*n >= 1 somewhere, or tau <= 1/2           */
};

typedef struct lbm_solver lbm_solver; /* opaque, owned by the library */
typedef struct lbm_batch lbm_batch;   /* opaque, owned by the library */

typedef struct {
    int32_t nx, ny, nz; /* structure size in voxels (x is the transport direction) */
    double voxel_m;     /* voxel edge in metres (Knudsen diffusivity, Eq. 8)       */
} lbm_grid;

typedef struct {
    uint32_t struct_size;      /* = sizeof(lbm_params); guards against ABI drift    */
    int32_t mode;              /* LBM_MODE_*                                        */
    double c_in, c_out;        /* Dirichlet values at x = 0 and x = L (c_out unused
                                  in LBM_MODE_REACT, whose outlet is zero-gradient) */
    double tau_ref;            /* relaxation time given to D_ref (default 1)        */
    double w0;                 /* D3Q7 rest weight (default 1/4)                    */
    int32_t knudsen;           /* 1: pore D by Bosanquet with local Knudsen D       */
    double T_K, p_atm, M_kg_mol; /* temperature, pressure, molar mass (353, 1, 0.032) */
    double d_ionomer_rel;      /* ionomer D / D0 (default 1e-3)                     */
    double d_ref_rel;          /* 0: D_ref = largest simulated D; else D_ref/D0     */
    double k_lat;              /* first-order rate per catalyst face, lattice units */
    uint32_t catalyst_phases;  /* bit mask over phase ids (default 1 << LBM_PT)     */
    uint32_t reactive_fluids;  /* bit mask of fluid phases that react (pore|ionomer)*/
    int32_t reservoir_plane;   /* REACT: prepend one pore plane at the inlet (1)    */
    double tol_change;         /* stop: max|C_t - C_{t-K}| / (K max|C|) below this  */
    double tol_flux;           /* stop: estimated remaining relative error of the
                                  output (flux or rate) and of the total mass below
                                  this (default 1e-5)                               */
    double tol_balance;        /* stop: |J_in - J_out - R| / |J_in| below this      */
    int32_t check_every;       /* K: steps between convergence checks (even)        */
    int64_t max_steps;         /* give up (LBM_NOT_CONVERGED) after this many steps */
} lbm_params;

typedef struct {
    int64_t steps;      /* LBM steps taken since the last initialisation          */
    double residual;    /* max|C_t - C_{t-K}| / (K max|C_t|) at the last check    */
    double j_in;        /* net flux through the inlet face, per unit area         */
    double j_out;       /* net flux through the outlet face, per unit area        */
    double j_vol;       /* net x flux averaged over all interior faces, per area  */
    double rate;        /* total sink sum k n C, per unit cross-section area      */
    double mass;        /* total sum of C over simulated voxels                   */
    double est_error;   /* estimated remaining relative error of the output       */
    double kernel_ms;   /* HIP-event time of the stream-collide launches made by
                           the steady-state loop since the last initialisation    */
    int64_t kernel_launches; /* steps timed in kernel_ms (a two-step launch: 2)  */
    int32_t status;     /* LBM_OK, LBM_NOT_CONVERGED or an error                  */
    int32_t checks;     /* number of convergence checks made                      */
} lbm_run_info;

typedef struct {
    int32_t nx, ny, nz;    /* simulated grid (REACT with reservoir: nx + 1)       */
    int32_t nx_struct;     /* structure size along x                              */
    int64_t n_active;      /* simulated voxels (transport, connected)             */
    int64_t n_segments;    /* segments: windows of up to 64 voxels consecutive in
                              grid order, each row cut into its own windows, or
                              (rows of 64 k + 1 voxels) windows running on across
                              row ends within a plane                              */
    double d0;             /* D0 (m^2/s; 1 in proton mode)                        */
    double d_ref;          /* D_ref (same units)                                  */
    double d0_lat;         /* D0 in lattice units                                 */
    int32_t percolates;    /* transport path joins the Dirichlet faces            */
    int32_t mode;
    int64_t n_listed;      /* segments holding simulated voxels: the waves of one
                              stream-collide launch                                */
} lbm_info;

/* Fill *p with the defaults listed above.  Returns LBM_ERR_INVALID_ARG on NULL. */
int lbm_params_default(lbm_params *p);

/* Preprocess a structure (host only, no device call): phases -> transport mask,
 * 13-direction pore size (Section 2.1.3), local D (Eqs. 7-9, 15), tau (Eq. 24),
 * catalyst neighbour counts (Eq. 18a), dead-pocket removal, and the segment
 * bitmasks used by the kernels.  phase_host is nz*ny*nx bytes, copied.  On
 * success *out receives a new handle.  Errors: INVALID_ARG, BAD_PHASE, UNSTABLE. */
int lbm_create(const lbm_grid *g, const uint8_t *phase_host, const lbm_params *p, lbm_solver **out);

/* lbm_create with the device's share of the preprocessing: the two steps whose
 * cost grows with the voxel count, the 13-direction pore size (Section 2.1.3) and
 * the reach of the transport phases from the Dirichlet faces, run on the current
 * device (as lbm_pore_size_device and lbm_reach_device) instead of the host.  Every
 * other step, and every result (the handle's host fields included), is that of
 * lbm_create, bit for bit.  scratch_dev: caller-owned device memory of at least
 * lbm_prep_scratch_bytes bytes, 256-byte aligned, free for other use again when
 * the call returns; stream: a hipStream_t (NULL: the null stream), synchronised
 * before the call returns.  Errors: those of lbm_create, LBM_ERR_WORKSPACE for a
 * missing, small or misaligned scratch, LBM_ERR_HIP for a failed device call
 * (lbm_last_error names it).
 * lbm_batch_create_device is the same for lbm_batch_create: instances are
 * prepared on parallel host threads that take turns on the device.
 * lbm_prep_scratch_bytes: the scratch these calls need for n structures (the
 * largest instance's: about 10 bytes per voxel). */
int lbm_prep_scratch_bytes(int32_t n, const lbm_grid *grids, const lbm_params *params, size_t *bytes);
int lbm_create_device(const lbm_grid *g, const uint8_t *phase_host, const lbm_params *p, void *scratch_dev,
                      size_t scratch_bytes, void *stream, lbm_solver **out);

/* Sizes and reference values of a created solver. */
int lbm_get_info(const lbm_solver *s, lbm_info *info);

/* Host copies of the preprocessed fields on the simulated grid (dense, N bytes or
 * floats each).  Any pointer may be NULL.  active: 1 for simulated voxels;
 * n_cat: catalyst face-neighbour count (0..6) of every voxel; omega: 1/tau of
 * simulated voxels (FP32 as used on the device), 0 elsewhere. */
int lbm_get_host_fields(const lbm_solver *s, uint8_t *active_host, uint8_t *n_cat_host, float *omega_host);

/* Structure descriptor used by the learned warm start (not part of the paper's
 * method): for every voxel of the simulated grid (N bytes, host), the number of
 * 6-neighbour steps through simulated voxels (periodic in y and z) from the pore
 * voxels joined to a Dirichlet face through pore voxels alone.  0 on those pores,
 * 1..254 beyond them (ionomer films, pore pockets reached only through ionomer),
 * 255 for voxels that are not simulated, farther than 254 steps or unreached.
 * Computed on the host on each call (O(N)). */
int lbm_get_pore_depth(const lbm_solver *s, uint8_t *depth_host);

/* Device bytes the solver needs (distributions, metadata, reduction scratch). */
int lbm_workspace_bytes(const lbm_solver *s, size_t *bytes);

/* Hand the solver a device workspace (>= lbm_workspace_bytes, 256-byte aligned)
 * and a HIP stream (hipStream_t, may be NULL for the default stream).  Uploads the
 * metadata and initialises the distributions to equilibrium at C = c_out (REACT:
 * C = 0).  Errors: INVALID_ARG, WORKSPACE, HIP. */
int lbm_bind(lbm_solver *s, void *workspace_dev, size_t bytes, void *hip_stream);

/* Initialise the distributions to equilibrium f_i = w_i C (Eq. 23) from a dense
 * FP32 concentration field on the simulated grid (NULL: cold start as in
 * lbm_bind).  Resets the step count and the convergence history. */
int lbm_set_initial_concentration(lbm_solver *s, const float *c_dev);

/* Set the stored post-collision distributions from a dense FP32 [7][N] array on
 * the simulated grid (values of non-simulated voxels are ignored). */
int lbm_set_populations(lbm_solver *s, const float *f_dev);

/* Copy the stored post-collision distributions to a dense FP32 [7][N] array
 * (non-simulated voxels receive 0).  The values are the unshifted f_i = g_i +
 * w_i c_sh(x), each rounded once to FP32 from the stored FP32 g_i, so writing them
 * back with lbm_set_populations reproduces the stored state only up to that
 * rounding. */
int lbm_get_populations(const lbm_solver *s, float *f_dev);

/* Advance nsteps >= 0 fused stream-collide steps (Eq. 21) without checks. */
int lbm_step(lbm_solver *s, int64_t nsteps);

/* FP64 reductions of the current state (no stepping): the fluxes of the next
 * streaming, the sink and the mass, exactly as the steady-state outputs use them.
 * Fills j_in, j_out, j_vol, rate, mass; leaves the convergence fields alone. */
int lbm_measure(lbm_solver *s, lbm_run_info *info);

/* Step to the steady state.  Checks follow windows of K steps (doubled while the
 * mass of some live instance still decays by less than half per window); the run stops when the windowed
 * residual, the estimated remaining relative error of the output and of the total
 * mass (geometric extrapolation with the decay rate measured on the mass), and the
 * flux balance are all below their tolerances, or after max_steps.  A window
 * never exceeds 1/32 of the steps already taken.  Returns LBM_OK, LBM_NOT_CONVERGED,
 * LBM_ERR_DIVERGED or LBM_ERR_NO_PERCOLATION (D_eff problems without a path). */
int lbm_run_to_steady(lbm_solver *s, lbm_run_info *info);

/* Tiling of the stream-collide launch: segments per wave (1, 2, 4), waves per
 * workgroup (1, 2, 4, 8), XCD-aware workgroup order (0/1).  lbm_autotune times
 * every tiling, and every two-step form below, for steps_per_trial steps on the
 * live state (the trial steps are ordinary solver steps) and keeps the fastest;
 * ms_best receives its time per step. */
int lbm_set_tiling(lbm_solver *s, int32_t segs_per_wave, int32_t waves_per_block, int32_t xcd_remap);
int lbm_get_tiling(const lbm_solver *s, int32_t *segs_per_wave, int32_t *waves_per_block, int32_t *xcd_remap);
int lbm_autotune(lbm_solver *s, int32_t steps_per_trial, double *ms_best);

/* Two time steps per stream-collide launch (temporal blocking, Section 4's update
 * applied twice with the intermediate populations kept on chip).  A workgroup owns
 * one 64-voxel x range and rows_per_tile rows in y (4, 6 or 8) and marches through
 * planes_per_chunk planes in z (1 .. 64); the populations between the two steps
 * are rounded to FP32 exactly as a stored lattice is, so the results are
 * bit-identical to two single-step launches.  rows_per_tile 0 returns to one step
 * per launch (the default); an odd step count ends with one single-step launch.
 * Returns LBM_ERR_INVALID_ARG for other values, and for rows_per_tile > 0 on a
 * grid whose rows are 64 k + 1 voxels long (its segments run across row ends,
 * see lbm_info.n_segments; the tiles need each row cut into its own). */
int lbm_set_temporal(lbm_solver *s, int32_t rows_per_tile, int32_t planes_per_chunk);
int lbm_get_temporal(const lbm_solver *s, int32_t *rows_per_tile, int32_t *planes_per_chunk);

/* The loop of lbm_run_to_steady with a budget: at most max_new_steps further
 * steps (whole windows of K steps; fewer than K steps of budget does nothing).
 * Returns LBM_OK once converged, LBM_NOT_CONVERGED while the budget ran out
 * first (call again to continue), or an error. */
int lbm_advance(lbm_solver *s, int64_t max_new_steps, lbm_run_info *info);

/* D_eff/D0 (LBM_MODE_DEFF) or sigma_eff/sigma (LBM_MODE_PROTON) from the volume
 * averaged x flux of the last measurement, Eq. (19) with L = nx:
 * J * nx / ((c_in - c_out) * D0_lat).  WRONG_MODE in LBM_MODE_REACT. */
int lbm_deff(const lbm_solver *s, double *deff_over_d0);

/* Total reaction rate per unit cross-section area (sum k n C / (ny nz)) and the
 * inlet flux per unit area (lattice units), LBM_MODE_REACT only. */
int lbm_reaction_rate(const lbm_solver *s, double *rate_per_area, double *j_in);

/* Dense FP32 concentration on the simulated grid (0 off the simulated voxels). */
int lbm_concentration(const lbm_solver *s, float *c_dev);

/* Release the handle (NULL is a no-op). The workspace stays the caller's. */
void lbm_destroy(lbm_solver *s);

/* Static text for a status code. */
const char *lbm_status_string(int status);

/* Text naming the first HIP call that failed in the calling thread's last failing
 * operation ("" if none); valid until the next call on this thread. */
const char *lbm_last_error(void);

/* ---------------------------------------------------------------- batched form
 * Many independent structures of uneven size in one launch per step, captured in
 * a HIP graph, with per-instance FP64 reductions and retirement at check
 * boundaries.  All instances share mode and the Knudsen switch; every other
 * parameter (k, c_in, tau_ref, ...) is per instance. */

/* n >= 1 structures; grids[i], phases_host[i] (nz*ny*nx bytes), params[i]. */
int lbm_batch_create(int32_t n, const lbm_grid *grids, const uint8_t *const *phases_host,
                     const lbm_params *params, lbm_batch **out);
/* lbm_batch_create with the device's share of the preprocessing (see lbm_create_device). */
int lbm_batch_create_device(int32_t n, const lbm_grid *grids, const uint8_t *const *phases_host,
                            const lbm_params *params, void *scratch_dev, size_t scratch_bytes, void *stream,
                            lbm_batch **out);
int lbm_batch_workspace_bytes(const lbm_batch *b, size_t *bytes);
int lbm_batch_bind(lbm_batch *b, void *workspace_dev, size_t bytes, void *hip_stream);
/* Tiling chosen by lbm_batch_autotune (or set explicitly): segments per wave
 * (1, 2, 4), waves per workgroup (1, 2, 4, 8), XCD-aware block order (0/1). */
int lbm_batch_set_tiling(lbm_batch *b, int32_t segs_per_wave, int32_t waves_per_block, int32_t xcd_remap);
int lbm_batch_get_tiling(const lbm_batch *b, int32_t *segs_per_wave, int32_t *waves_per_block, int32_t *xcd_remap);
/* Time every tiling on the live workload (steps_per_trial steps each, state is
 * restored afterwards) and keep the fastest; ms_best receives its time per step. */
int lbm_batch_autotune(lbm_batch *b, int32_t steps_per_trial, double *ms_best);
/* Run all instances to their steady states; infos[n] receives per-instance results. */
int lbm_batch_run(lbm_batch *b, lbm_run_info *infos);
/* As lbm_batch_run, but stop once max_new_steps more steps have been taken (check
 * windows are shortened to fit).  Finished instances stay finished; the others
 * report LBM_NOT_CONVERGED and continue from where they are on the next call.
 * Returns the worst status, LBM_NOT_CONVERGED while any instance is running. */
int lbm_batch_advance(lbm_batch *b, int64_t max_new_steps, lbm_run_info *infos);
/* lbm_batch_run and lbm_batch_advance take the pending instances in groups whose
 * combined working set (both lattices, 1/tau, snapshot and segment records: about
 * 64 bytes per simulated voxel) stays within this many bytes, one group after the
 * other, so each group stays resident in the GPU's 256 MB last-level cache while
 * it steps.  Default 192 MiB; 0 runs every instance together. */
int lbm_batch_set_group_bytes(lbm_batch *b, int64_t bytes);
int lbm_batch_deff(const lbm_batch *b, int32_t i, double *deff_over_d0);
int lbm_batch_reaction_rate(const lbm_batch *b, int32_t i, double *rate_per_area, double *j_in);
int lbm_batch_get_info(const lbm_batch *b, int32_t i, lbm_info *info);
/* Instance i's dense FP32 concentration on its own simulated grid (device) and
 * its preprocessed host fields (as lbm_get_host_fields). */
int lbm_batch_concentration(const lbm_batch *b, int32_t i, float *c_dev);
/* Instance i's pore-depth map (as lbm_get_pore_depth). */
int lbm_batch_get_pore_depth(const lbm_batch *b, int32_t i, uint8_t *depth_host);
int lbm_batch_get_host_fields(const lbm_batch *b, int32_t i, uint8_t *active_host, uint8_t *n_cat_host,
                              float *omega_host);
void lbm_batch_destroy(lbm_batch *b);

/* ---- Structure characterisation on the device (Section 2.1.3)
 *
 * The two preprocessing steps whose cost grows with the voxel count, for phase
 * maps already in device memory.  Arrays are device pointers to nz*ny*nx voxels,
 * x fastest; y and z are periodic and x is bounded, as in lbm_create.  stream is
 * a hipStream_t (NULL: the null stream); both calls synchronise it before
 * returning.  Errors: LBM_ERR_INVALID_ARG for NULL pointers, non-positive sizes
 * or (reach) faces outside 1..3; LBM_ERR_HIP for a failed launch (lbm_last_error
 * names it).
 *
 * lbm_pore_size_device: the pore size of Section 2.1.3 (the d_p of Eqs. 8-9, in
 * voxel edges).  For a voxel with pore_dev[v] != 0, dp_dev[v] (FP64) is the mean
 * over the 13 directions d of the length, in voxels, of the run of pore voxels
 * through v along d, times |d|. A run along a direction without an x component
 * that closes on itself under the wrap counts its loop once. Other voxels get 0.
 * The sum runs in lbm_create's direction order with round-to-nearest products
 * and sums, so the values are bit-identical to the host's.
 *
 * lbm_reach_device: hit_dev[v] = 1 for every voxel with pass_dev[v] != 0 that is
 * 6-neighbour connected through such voxels to one on the x = 0 face (faces & 1)
 * or the x = nx - 1 face (faces & 2); 0 elsewhere.  This is lbm_create's
 * simulated-voxel mask when pass is the transport phase and faces are the
 * Dirichlet faces.  *cycles (may be NULL) receives the number of sweep cycles
 * (three line sweeps each) until nothing changed. */
int lbm_pore_size_device(const uint8_t *pore_dev, int32_t nx, int32_t ny, int32_t nz, double *dp_dev, void *stream);
int lbm_reach_device(const uint8_t *pass_dev, int32_t nx, int32_t ny, int32_t nz, int32_t faces, uint8_t *hit_dev,
                     int32_t *cycles, void *stream);

/* lbm_reach_device_static: lbm_reach_device for callers that cannot allocate
 * (code under HIP graph capture elsewhere on the stream's device, tight serving
 * loops, harnesses that forbid allocation).  Same arguments, results and errors;
 * it calls no hipMalloc, hipHostMalloc or other allocating routine.  The sweeps'
 * change flag lives in a fixed 256-byte device array of this library (one copy per
 * device, held until the process ends) instead of freshly allocated pinned host
 * memory; it does not grow with the grid, so every grid lbm_reach_device accepts
 * is accepted.  The flag is cleared by a kernel at the start of every sweep cycle
 * and read back with a copy into host memory followed by a synchronisation of
 * stream, once per cycle.  Calls that overlap on one device (other host threads,
 * other streams) share that flag and race: serialise them. */
int lbm_reach_device_static(const uint8_t *pass_dev, int32_t nx, int32_t ny, int32_t nz, int32_t faces,
                            uint8_t *hit_dev, int32_t *cycles, void *stream);

/* ---- D3Q19 solver (Section 4, Eqs. 21-24: the paper's own lattice)
 *
 * The same problems as lbm_create (modes, phases, Knudsen diffusivity, sink,
 * boundary conditions of Section 3.5, stop rule parameters) on the 19-velocity
 * lattice of Eq. (22) with the weights of Eq. (23): a_0 = 1/3, 1/18 for the six
 * face velocities, 1/36 for the twelve edge velocities, c_s^2 = 1/3 and
 * D = (tau - 1/2)/3 in lattice units (Eq. 24).  lbm_params.w0 is ignored.
 *
 * Direction order (the populations' order in device arrays): 0 rest; 1 +x,
 * 2 -x, 3 +y, 4 -y, 5 +z, 6 -z; 7..10 (x,y) = (+,+), (+,-), (-,+), (-,-);
 * 11..14 (x,z) in the same pattern; 15..18 (y,z) in the same pattern.
 *
 * Boundaries: half-way bounce-back toward voxels that are not simulated;
 * periodic y and z; at x = 0 (and at x = nx - 1 outside LBM_MODE_REACT) a
 * population entering from the reservoir takes the anti-bounce-back Dirichlet
 * value when the voxel of the face plane it passes (shifted by its y and z
 * components) is simulated, and bounces back otherwise.  The reactive outlet is
 * zero-gradient (bounce-back).
 *
 * Memory: dense over the simulated grid.  lbm19_workspace_bytes gives the size
 * of the caller-owned device workspace: two FP32 lattices of 19 planes of N
 * values (each plane padded by at most 4.5 KB), 16 N bytes of per-voxel data
 * and small reduction buffers, N = nx ny nz of the simulated grid.
 * lbm19_bind takes it (256-byte aligned) with a hipStream_t (NULL: the null
 * stream) on which all work is queued, uploads the per-voxel data and sets the
 * cold start (C = 0).  The workspace must outlive the solver's
 * use of it.  Calls that return host values synchronise the stream.  One solver
 * per thread.
 *
 * lbm19_create: as lbm_create.  Also LBM_ERR_INVALID_ARG when one lattice would
 *   reach 4 GiB (more than about 56 million simulated voxels, ~383^3).
 * lbm19_set_initial_concentration: stored state f_i = a_i C0 with C0 a device
 *   FP32 array of N values (NULL: C0 = 0); resets the step count.
 * lbm19_step: nsteps steps of Eq. (21).
 * lbm19_measure: one step that also measures; *info (may be NULL) receives the
 *   fluxes of the links crossed during that step (j_in, j_out, j_vol per unit
 *   area), rate and mass of the new state; LBM_ERR_DIVERGED on NaN.
 * lbm19_run_to_steady: windows of check_every steps; stops when max|dC| per step
 *   over a window is below tol_change max|C|, the output (j_vol, or the rate
 *   when reacting) is within tol_flux of its limit as estimated from the ratio
 *   of successive window changes, on two checks in a row, and
 *   |J_in - J_out - R| <= tol_balance |J_in|; LBM_NOT_CONVERGED at max_steps;
 *   LBM_ERR_NO_PERCOLATION at once when no transport path joins the Dirichlet
 *   faces.  kernel_ms and kernel_launches are not filled.
 * lbm19_deff / lbm19_reaction_rate: as lbm_deff / lbm_reaction_rate, from the
 *   last measurement, with D0 in lattice units (tau_ref - 1/2) D0 / (3 D_ref).
 * lbm19_get_populations: f_dev (device, FP64, 19 N values in the direction
 *   order above, x fastest) receives the unshifted post-collision populations of
 *   the current state; 0 off the simulated voxels.
 * lbm19_concentration: c_dev (device, FP32, N values) receives C of the current
 *   state; 0 off the simulated voxels.
 * lbm19_get_info: as lbm_get_info (n_segments = 0). */
typedef struct lbm19_solver lbm19_solver;
int lbm19_create(const lbm_grid *g, const uint8_t *phase_host, const lbm_params *p, lbm19_solver **out);
int lbm19_get_info(const lbm19_solver *s, lbm_info *info);
int lbm19_workspace_bytes(const lbm19_solver *s, size_t *bytes);
int lbm19_bind(lbm19_solver *s, void *workspace_dev, size_t bytes, void *hip_stream);
int lbm19_set_initial_concentration(lbm19_solver *s, const float *c_dev);
int lbm19_step(lbm19_solver *s, int64_t nsteps);
int lbm19_measure(lbm19_solver *s, lbm_run_info *info);
int lbm19_run_to_steady(lbm19_solver *s, lbm_run_info *info);
int lbm19_deff(const lbm19_solver *s, double *deff_over_d0);
int lbm19_reaction_rate(const lbm19_solver *s, double *rate_per_area, double *j_in);
int lbm19_get_populations(const lbm19_solver *s, double *f_dev);
int lbm19_concentration(const lbm19_solver *s, float *c_dev);
void lbm19_destroy(lbm19_solver *s);

/* ---- Coupled oxygen / proton-potential problem on D3Q19 (Sections 3.2-3.4,
 * Eqs. 15-18b with the Tafel rate of Eq. 17b)
 *
 * Two D3Q19 solvers on one structure, coupled by Picard iteration on the device:
 *   O2: the reactive problem of lbm19_create (p->mode must be LBM_MODE_REACT;
 *       reservoir plane, inlet C_in, zero-gradient outlet) whose sink sits on the
 *       reaction sites only, with k n = k_ref n exp(beta (phi - phi_ref));
 *   potential: D_phi lap(phi) = q on the ionomer joined to the membrane face
 *       x = L through ionomer, phi = phi_m there (anti-bounce-back), zero proton
 *       flux at x = 0 and every other boundary, D_phi from tau_phi, with the
 *       proton source q = gamma n (C / C_in) exp(beta (phi - phi_ref)) (Eq. 18b).
 * Reaction sites: ionomer voxels with n > 0 Pt face neighbours that both
 * problems reach.  From phi = phi_m: solve O2, then the potential, then move phi
 * by theta of the change; stop when the change is below tol_phi (volts) on every
 * voxel (LBM_OK) or after max_iter iterations (LBM_NOT_CONVERGED).  Each inner
 * solve is lbm19_run_to_steady with p's stop parameters, continuing from the
 * previous iterate.  The paper itself presets a uniform phi (Section 3.5.2); the
 * boundary values above are this library's reading, documented with the oracle.
 *
 * lbm_coupling_default: k_ref 1e-2, beta 21.3 1/V (alpha F / R T at alpha 0.61,
 *   333 K), gamma 1e-3 V, phi_m = phi_ref = 0.6 V, tau_phi 1, theta 0.5,
 *   tol_phi 1e-6 V, max_iter 200, potential_solver 0.
 * Potential solves: at tau_phi = 1 every post-collision population of the
 *   potential lattice is a_i u with u = phi + S, so its steady state is the
 *   solution of sum_links a_i (u(x) - u(x - c_i)) + sum_open 2 a_i (u(x) - phi_m)
 *   = S(x) (links to simulated voxels; open links at the membrane face).  With
 *   potential_solver 0 that symmetric positive definite system is solved on the
 *   device by Jacobi-preconditioned conjugate gradients in FP64 to a residual of
 *   1e-12 of the right-hand side, starting from the previous iterate, and the
 *   lattice is set to the equilibrium a_i u, followed by one measured step; with
 *   1 (or tau_phi != 1) the lattice steps to its own stop rule.
 * lbm19_coupled_create: LBM_ERR_INVALID_ARG for NULL pointers, a struct_size
 *   mismatch, k_ref <= 0, beta < 0, gamma < 0, tau_phi <= 1/2, theta outside
 *   (0, 1], tol_phi <= 0, max_iter < 1, a mode other than LBM_MODE_REACT or
 *   c_in <= 0; LBM_ERR_UNSTABLE when 6 k_ref exp(beta max(0, phi_m - phi_ref))
 *   >= 1; LBM_ERR_NO_PERCOLATION when no reaction site is reached by both
 *   problems; otherwise the errors of lbm19_create.
 * lbm19_coupled_workspace_bytes / lbm19_coupled_bind: as lbm19_*; the workspace
 *   holds both solvers and five FP32 fields of the structure grid.
 * lbm19_coupled_run: the iteration above; *info (may be NULL) receives the
 *   iteration count, the last change of phi, the lowest phi, the O2 consumption
 *   and the proton source per unit area, the membrane current per unit area and
 *   the step counts of the two solvers.
 * lbm19_coupled_fields: c_dev (O2 grid, reservoir plane included) and phi_dev
 *   (structure grid; phi_m off the potential's voxels), device FP32; either may
 *   be NULL. */
typedef struct {
    uint32_t struct_size; /* = sizeof(lbm_coupling)                              */
    double k_ref;         /* O2 rate per Pt face at phi_ref, lattice units       */
    double beta;          /* alpha F / (R T), 1/V                                */
    double gamma;         /* proton source per Pt face at C_in and phi_ref, V    */
    double phi_m;         /* potential at the membrane face x = L, V             */
    double phi_ref;       /* potential at which k_ref and gamma hold, V          */
    double tau_phi;       /* relaxation time of the potential lattice            */
    double theta;         /* Picard under-relaxation, (0, 1]                     */
    double tol_phi;       /* stop when phi changes by less than this, V          */
    int32_t max_iter;
    int32_t potential_solver; /* 0: at tau_phi = 1 the potential's steady state by
                                 conjugate gradients on its exact equivalent (the
                                 D3Q19 link Laplacian), else by stepping; 1: always
                                 by stepping the potential lattice                */
} lbm_coupling;

typedef struct {
    int32_t iterations, status;
    double dphi;          /* last change of phi, V                               */
    double phi_min;       /* lowest phi, V                                       */
    double rate;          /* O2 consumption per unit area (sum k n C / A)        */
    double source;        /* proton source per unit area (sum q / A)             */
    double proton_in;     /* current in through the membrane face, per area      */
    int64_t o2_steps, phi_steps;
    int64_t phi_cg_iterations; /* conjugate-gradient iterations of all potential solves */
} lbm_coupled_info;

typedef struct lbm19_coupled lbm19_coupled;
int lbm_coupling_default(lbm_coupling *c);
int lbm19_coupled_create(const lbm_grid *g, const uint8_t *phase_host, const lbm_params *p, const lbm_coupling *cp,
                         lbm19_coupled **out);
int lbm19_coupled_workspace_bytes(const lbm19_coupled *c, size_t *bytes);
int lbm19_coupled_bind(lbm19_coupled *c, void *workspace_dev, size_t bytes, void *hip_stream);
int lbm19_coupled_run(lbm19_coupled *c, lbm_coupled_info *info);
int lbm19_coupled_fields(const lbm19_coupled *c, float *c_dev, float *phi_dev);
void lbm19_coupled_destroy(lbm19_coupled *c);

#ifdef __cplusplus
}
#endif
#endif
