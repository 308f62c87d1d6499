/*
 * Plain FP64 reference ("oracle") for the D3Q7 single-relaxation-time lattice
 * Boltzmann model of steady diffusion with a first-order sink, after Chen et al.,
 * "Nanoscale study of reactive transport in catalyst layer of PEMFC ... using the
 * lattice Boltzmann method" (arXiv 1410.1914), Section 4, Eqs. (21)-(24), with the
 * boundary conditions of Section 3.5 (Eqs. 19, 20a, 20b).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference for the HIP
 * solver.  Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header or constant table with the
 * product library, and it includes nothing from it.
 *
 * Everything here is deliberately plain: dense arrays, one loop per step of the
 * method, no blocking, no fusion, FP64 throughout.
 *
 * Layout: every field is dense over the simulated grid, voxel index
 * v = (z*ny + y)*nx + x (x fastest).  Populations are f[i*N + v], i = 0..6 in the
 * order rest, +x, -x, +y, -y, +z, -z.
 *
 * The caller (oracle/lbm.py) supplies the per-voxel fields that Section 3 defines:
 *   active[v]  1 if the voxel is a transport voxel connected to a Dirichlet face
 *   omega[v]   1/tau, tau from the local diffusivity (Eq. 24)
 *   kn[v]      k * n(v), the first-order sink coefficient (Eqs. 17b, 18a)
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* threads the parallel loops below use (1 without OpenMP) */
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static const int CX[7] = {0, 1, -1, 0, 0, 0, 0};
static const int CY[7] = {0, 0, 0, 1, -1, 0, 0};
static const int CZ[7] = {0, 0, 0, 0, 0, 1, -1};
static const int OPP[7] = {0, 2, 1, 4, 3, 6, 5};

typedef struct {
    int32_t nx, ny, nz;
    int32_t react;      /* 1: zero-gradient outlet (Eq. 20a); 0: Dirichlet outlet */
    double c_in, c_out; /* Dirichlet values at the x = 0 and x = nx faces          */
    double w0;          /* rest weight; moving weights are (1 - w0) / 6           */
    const uint8_t *active;
    const double *omega;
    const double *kn;
} orc_grid;

static double weight(const orc_grid *g, int i) { return i == 0 ? g->w0 : (1.0 - g->w0) / 6.0; }

static int64_t vid(const orc_grid *g, int x, int y, int z) {
    return ((int64_t)z * g->ny + y) * g->nx + x;
}

/* Collision with source, Eq. (21) right-hand side: g* = g - (g - g_eq)/tau + w_i S,
 * g_eq = w_i C (Eq. 23 read as w_i * C), C = sum_i g_i (Eq. 24), S = -k n C. */
void orc_collide(const orc_grid *g, const double *f, double *fs) {
    const int64_t N = (int64_t)g->nx * g->ny * g->nz;
    memset(fs, 0, sizeof(double) * 7 * N);
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < N; ++v) {
        if (!g->active[v]) continue;
        double C = 0.0;
        for (int i = 0; i < 7; ++i) C += f[i * N + v];
        const double S = -g->kn[v] * C;
        for (int i = 0; i < 7; ++i) {
            const double w = weight(g, i);
            fs[i * N + v] = f[i * N + v] - g->omega[v] * (f[i * N + v] - w * C) + w * S;
        }
    }
}

/* Streaming, Eq. (21) left-hand side, with the boundary rules of Section 3.5:
 * periodic y and z; half-way bounce-back where the target is impermeable;
 * anti-bounce-back Dirichlet at the x faces (C_in at x = 0, C_out at x = nx in the
 * effective-property problems); plain bounce-back (zero gradient) at x = nx in the
 * reactive problem. */
void orc_stream(const orc_grid *g, const double *fs, double *f) {
    const int64_t N = (int64_t)g->nx * g->ny * g->nz;
    memset(f, 0, sizeof(double) * 7 * N);
    /* every (voxel, direction) slot of an active voxel is written exactly once,
     * so the planes can be processed in parallel */
#pragma omp parallel for schedule(static)
    for (int z = 0; z < g->nz; ++z)
        for (int y = 0; y < g->ny; ++y)
            for (int x = 0; x < g->nx; ++x) {
                const int64_t v = vid(g, x, y, z);
                if (!g->active[v]) continue;
                for (int i = 0; i < 7; ++i) {
                    const double val = fs[i * N + v];
                    const int tx = x + CX[i];
                    const int ty = ((y + CY[i]) % g->ny + g->ny) % g->ny;
                    const int tz = ((z + CZ[i]) % g->nz + g->nz) % g->nz;
                    const double w = weight(g, i);
                    if (tx < 0) {
                        f[OPP[i] * N + v] = -val + 2.0 * w * g->c_in;
                    } else if (tx >= g->nx) {
                        f[OPP[i] * N + v] = g->react ? val : -val + 2.0 * w * g->c_out;
                    } else {
                        const int64_t t = vid(g, tx, ty, tz);
                        if (g->active[t])
                            f[i * N + t] = val;
                        else
                            f[OPP[i] * N + v] = val;
                    }
                }
            }
}

/* One time step in the order of Eq. (21): collide, then stream.  tmp holds 7N. */
void orc_step(const orc_grid *g, const double *f, double *fnew, double *tmp) {
    orc_collide(g, f, tmp);
    orc_stream(g, tmp, fnew);
}

/* Concentration C = sum_i f_i on every voxel (0 where inactive). */
void orc_concentration(const orc_grid *g, const double *f, double *C) {
    const int64_t N = (int64_t)g->nx * g->ny * g->nz;
    for (int64_t v = 0; v < N; ++v) {
        double s = 0.0;
        if (g->active[v])
            for (int i = 0; i < 7; ++i) s += f[i * N + v];
        C[v] = s;
    }
}

/* Fluxes of the streaming that follows the state f (pre-collision populations).
 * out[0] = J_in   net flux entering through the x = 0 face
 * out[1] = J_out  net flux leaving through the x = nx face
 * out[2] = sum over the nx-1 interior x faces of the net +x link flux
 * out[3] = R      total sink sum_v k n(v) C(v)
 * out[4] = M      total mass sum_v C(v)
 * All sums are totals (not per unit area).  face[p] (length nx-1, may be NULL)
 * receives the net flux through the face between planes p and p+1. */
void orc_fluxes(const orc_grid *g, const double *f, double *fs_scratch, double *out, double *face) {
    const int64_t N = (int64_t)g->nx * g->ny * g->nz;
    orc_collide(g, f, fs_scratch);
    const double *fs = fs_scratch;
    const double w1 = weight(g, 1);
    double jin = 0, jout = 0, jint = 0, R = 0, M = 0;
    for (int p = 0; p + 1 < g->nx; ++p)
        if (face) face[p] = 0.0;
    for (int z = 0; z < g->nz; ++z)
        for (int y = 0; y < g->ny; ++y)
            for (int x = 0; x < g->nx; ++x) {
                const int64_t v = vid(g, x, y, z);
                if (!g->active[v]) continue;
                double C = 0.0;
                for (int i = 0; i < 7; ++i) C += f[i * N + v];
                M += C;
                R += g->kn[v] * C;
                if (x == 0) jin += 2.0 * w1 * g->c_in - 2.0 * fs[2 * N + v];
                if (x == g->nx - 1 && !g->react) jout += 2.0 * fs[1 * N + v] - 2.0 * w1 * g->c_out;
                if (x + 1 < g->nx) {
                    const int64_t t = vid(g, x + 1, y, z);
                    if (g->active[t]) {
                        const double lf = fs[1 * N + v] - fs[2 * N + t];
                        jint += lf;
                        if (face) face[x] += lf;
                    }
                }
            }
    out[0] = jin;
    out[1] = jout;
    out[2] = jint;
    out[3] = R;
    out[4] = M;
}

/* The step is affine: f(t+1) = A f(t) + b.  Write A as COO triplets and b densely.
 * Row and column index = i*N + v.  Inactive voxels get no rows (their unknowns are
 * identically zero).  Capacity needed: 49 * (number of active voxels) triplets.
 * Returns the number of triplets written. */
int64_t orc_assemble(const orc_grid *g, int64_t *rows, int64_t *cols, double *vals, double *b) {
    const int64_t N = (int64_t)g->nx * g->ny * g->nz;
    int64_t k = 0;
    memset(b, 0, sizeof(double) * 7 * N);
    for (int z = 0; z < g->nz; ++z)
        for (int y = 0; y < g->ny; ++y)
            for (int x = 0; x < g->nx; ++x) {
                const int64_t v = vid(g, x, y, z);
                if (!g->active[v]) continue;
                const double om = g->omega[v], kn = g->kn[v];
                for (int i = 0; i < 7; ++i) {
                    /* destination of the post-collision population i of voxel v */
                    const int tx = x + CX[i];
                    const int ty = ((y + CY[i]) % g->ny + g->ny) % g->ny;
                    const int tz = ((z + CZ[i]) % g->nz + g->nz) % g->nz;
                    const double w = weight(g, i);
                    int64_t drow;
                    double sign = 1.0, cst = 0.0;
                    if (tx < 0) {
                        drow = OPP[i] * N + v;
                        sign = -1.0;
                        cst = 2.0 * w * g->c_in;
                    } else if (tx >= g->nx) {
                        drow = OPP[i] * N + v;
                        if (!g->react) {
                            sign = -1.0;
                            cst = 2.0 * w * g->c_out;
                        }
                    } else {
                        const int64_t t = vid(g, tx, ty, tz);
                        drow = g->active[t] ? i * N + t : OPP[i] * N + v;
                    }
                    /* post-collision population i as a combination of the 7 inputs */
                    for (int j = 0; j < 7; ++j) {
                        const double m = (i == j ? 1.0 - om : 0.0) + (om - kn) * w;
                        rows[k] = drow;
                        cols[k] = j * N + v;
                        vals[k] = sign * m;
                        ++k;
                    }
                    b[drow] += cst;
                }
            }
    return k;
}

/* Pore size by the 13-direction averaging method (Section 2.1.3): for every pore
 * voxel, along each of 13 lines through it, count the run of consecutive pore
 * voxels that contains it, convert the count to a length (count * |v|, in voxel
 * edges), and average the 13 lengths.  Lines wrap periodically in y and z (a run
 * is capped at the number of distinct voxels on the wrapped line) and stop at the
 * x faces.  dp[v] = 0 for non-pore voxels. */
static const int DIR13[13][3] = {{1, 0, 0},  {0, 1, 0},  {0, 0, 1}, {1, 1, 0}, {1, -1, 0},
                                 {1, 0, 1},  {1, 0, -1}, {0, 1, 1}, {0, 1, -1}, {1, 1, 1},
                                 {1, 1, -1}, {1, -1, 1}, {-1, 1, 1}};

/* number of distinct voxels visited by repeatedly stepping (dy, dz) with wrap */
static int64_t wrap_period(int ny, int nz, int dy, int dz) {
    int64_t y = 0, z = 0, n = 0;
    do {
        y = ((y + dy) % ny + ny) % ny;
        z = ((z + dz) % nz + nz) % nz;
        ++n;
    } while (y != 0 || z != 0);
    return n;
}

void orc_chords(int nx, int ny, int nz, const uint8_t *pore, double *dp) {
    const int64_t N = (int64_t)nx * ny * nz;
    for (int64_t v = 0; v < N; ++v) dp[v] = 0.0;
    /* voxels are independent: rows are shared out over threads, each voxel's sum is
       formed in the same order as in a serial loop */
#pragma omp parallel for collapse(2) schedule(dynamic, 4)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int64_t v = ((int64_t)z * ny + y) * nx + x;
                if (!pore[v]) continue;
                double sum = 0.0;
                for (int d = 0; d < 13; ++d) {
                    const int dx = DIR13[d][0], dy = DIR13[d][1], dz = DIR13[d][2];
                    /* a line with no x component is a closed loop; else bounded by x */
                    const int64_t cap = (dx == 0) ? wrap_period(ny, nz, dy, dz) : INT64_MAX;
                    int64_t count = 1;
                    for (int s = -1; s <= 1; s += 2) {
                        int cx = x, cy = y, cz = z;
                        for (;;) {
                            if (count >= cap) break;
                            cx += s * dx;
                            cy = ((cy + s * dy) % ny + ny) % ny;
                            cz = ((cz + s * dz) % nz + nz) % nz;
                            if (cx < 0 || cx >= nx) break;
                            if (!pore[((int64_t)cz * ny + cy) * nx + cx]) break;
                            ++count;
                        }
                    }
                    if (count > cap) count = cap;
                    sum += (double)count * sqrt((double)(dx * dx + dy * dy + dz * dz));
                }
                dp[v] = sum / 13.0;
            }
}

/* 6-connected flood fill over transport voxels from the seeds (periodic y, z).
 * reach[v] = 1 for every transport voxel reachable from a seed. */
void orc_flood(int nx, int ny, int nz, const uint8_t *transport, const uint8_t *seed, uint8_t *reach) {
    const int64_t N = (int64_t)nx * ny * nz;
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (N > 0 ? N : 1));
    int64_t head = 0, tail = 0;
    for (int64_t v = 0; v < N; ++v) {
        reach[v] = 0;
        if (transport[v] && seed[v]) {
            reach[v] = 1;
            queue[tail++] = v;
        }
    }
    while (head < tail) {
        const int64_t v = queue[head++];
        const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((int64_t)nx * ny));
        for (int i = 1; i < 7; ++i) {
            const int tx = x + CX[i];
            if (tx < 0 || tx >= nx) continue;
            const int ty = ((y + CY[i]) % ny + ny) % ny;
            const int tz = ((z + CZ[i]) % nz + nz) % nz;
            const int64_t t = ((int64_t)tz * ny + ty) * nx + tx;
            if (transport[t] && !reach[t]) {
                reach[t] = 1;
                queue[tail++] = t;
            }
        }
    }
    free(queue);
}
