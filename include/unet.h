/*
 * unet.h — C ABI of the learned warm start's kernels (gfx950).
 *
 * A 3-D U-Net predicts the steady concentration field of the reactive problem
 * (Chen et al., arXiv 1410.1914, Sections 3.4-3.5.2, Eqs. 15, 18a, 20a, 20b) from
 * the structure, and the lattice Boltzmann solver of lbm.h starts from that field
 * (equilibrium populations, Eq. 23) instead of from C = 0.  The network itself is
 * not part of the paper's method: it only changes the starting point, and the
 * converged answer is the solver's.
 *
 * Conventions
 *   - Activations and activation gradients are BF16 in NDHWC order (channel
 *     fastest): a[((z*ny + y)*nx + x)*ld + off + c].  ld is the channel stride of
 *     the buffer (a multiple of 8), off the first channel the call reads or writes,
 *     so two tensors can share one buffer (U-Net skip concatenation).
 *   - Channel counts of 3x3x3 convolutions are multiples of 16.
 *   - Weights are BF16 [cout][kpad] with k = tap * cin + ci, tap = (dz+1)*9 +
 *     (dy+1)*3 + (dx+1), zero beyond 27*cin up to kpad = unet_kpad(cin).  Weight
 *     gradients, biases, master weights and Adam moments are FP32.
 *   - Every pointer is device memory; every call enqueues on the given HIP stream
 *     and returns 0, or -1 on invalid arguments, -6 if the launch failed.
 *   - Zero padding at the domain boundary for 3x3x3 convolutions.
 */
#ifndef PAPER_1410_1914_AMD_UNET_H
#define PAPER_1410_1914_AMD_UNET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* padded K extent of a 3x3x3 convolution with cin input channels (multiple of 32) */
int32_t unet_kpad(int32_t cin);

/* y[v, off_y + co] = act(b[co] + sum_k W[co, k] x[v + tap(k), off_x + ci(k)]),
 * act = ReLU when relu != 0, else identity.  BF16 MFMA (16x16x32) with FP32
 * accumulation.  Output is BF16; when y32 is not NULL the FP32 result is also
 * written to y32[v * cout + co].  Activations are NDHWC rows of ldx / ldy
 * elements; cin and cout are multiples of 16, ldx, offx, ldy and offy multiples
 * of 8 (16-byte runs), x, w, y and y32 16-byte aligned, x and w each below 2 GiB,
 * else -1.  b may be NULL (no bias).  Each workgroup copies the input planes its
 * 4 x 64 voxels in three planes read (halo included) straight into LDS, 16
 * channels at a time, and keeps the weights of those channels in registers. */
int unet_conv3d_fwd(const uint16_t *x, int32_t ldx, int32_t offx, const uint16_t *w, const float *b,
                    uint16_t *y, int32_t ldy, int32_t offy, float *y32, int32_t nz, int32_t ny, int32_t nx,
                    int32_t cin, int32_t cout, int32_t relu, void *stream);

/* unet_conv3d_fwd over the concatenation of a full-resolution tensor and a
 * nearest-upsampled half-resolution one, without storing it: input channels
 * 0 .. cin1 - 1 are x (rows of ldx elements at offx on the nz x ny x nx grid) and
 * channels cin1 .. cin - 1 are x2 (rows of ldx2 at offx2 on the nz/2 x ny/2 x nx/2
 * grid; voxel (z, y, x) reads x2 at (z/2, y/2, x/2)).  This is the U-Net decoder's
 * input; the results equal unet_up_fwd into the rows of a concatenation followed by
 * unet_conv3d_fwd on them.  w is [cout][unet_kpad(cin)] over the concatenated
 * channels.  nz, ny and nx even, cin1 and cin - cin1 positive multiples of 16, x2
 * 16-byte aligned and below 2 GiB, ldx2 and offx2 multiples of 8; the rest as for
 * unet_conv3d_fwd; else -1. */
int unet_conv3d_fwd_cat(const uint16_t *x, int32_t ldx, int32_t offx, int32_t cin1, const uint16_t *x2,
                        int32_t ldx2, int32_t offx2, const uint16_t *w, const float *b, uint16_t *y, int32_t ldy,
                        int32_t offy, float *y32, int32_t nz, int32_t ny, int32_t nx, int32_t cin, int32_t cout,
                        int32_t relu, void *stream);

/* The network's last convolution and its head in one pass: y = ReLU(b + W * x)
 * (unet_conv3d_fwd with 16 input and 16 output channels), then out[v] = hb[0] +
 * base[v] + sum_c hw[c] y[v, c] on the BF16-rounded y, in channel order, as
 * unet_head_fwd forms it; y itself is not stored.  base may be NULL (zero); out is
 * FP32 per voxel.  The other requirements are unet_conv3d_fwd's; else -1. */
int unet_conv3d_fwd_head(const uint16_t *x, int32_t ldx, int32_t offx, const uint16_t *w, const float *b,
                         const float *hw, const float *hb, const float *base, float *out, int32_t nz, int32_t ny,
                         int32_t nx, void *stream);

/* Weights of the backward-data convolution: wt[ci, tap' * cout + co] =
 * w[co, (26 - tap') * cin + ci]; wt has kpad = unet_kpad(cout).  Running
 * unet_conv3d_fwd with wt (cin and cout swapped, no bias, no ReLU) on dy gives dx. */
int unet_conv3d_wtrans(const uint16_t *w, uint16_t *wt, int32_t cin, int32_t cout, void *stream);

/* dw[co, k] += sum_v dy[v, offdy + co] x[v + tap(k), offx + ci(k)] on BF16 MFMA
 * (16x16x32) with FP32 accumulation, and, when db is not NULL, db[co] += sum_v
 * dy[v, offdy + co].  dw is [cout][kpad] FP32.  cin and cout are multiples of 16;
 * ldx, offx, lddy, offdy multiples of 8 (16-byte loads), else -1. */
int unet_conv3d_wgrad(const uint16_t *x, int32_t ldx, int32_t offx, const uint16_t *dy, int32_t lddy, int32_t offdy,
                      int32_t nz, int32_t ny, int32_t nx, int32_t cin, int32_t cout, float *dw, float *db,
                      void *stream);

/* dpre[v, c] = dy[v, c] * (y[v, c] > 0) (ReLU backward, in place allowed) */
int unet_relu_bwd(const uint16_t *y, int32_t ldy, int32_t offy, uint16_t *dy, int32_t ldd, int32_t offd,
                  int64_t nvox, int32_t c, void *stream);

/* 2x2x2 average pooling (even sizes): y at (nz/2, ny/2, nx/2); backward adds
 * dy/8 into the eight children (accumulate into dx). */
int unet_pool_fwd(const uint16_t *x, int32_t ldx, int32_t offx, uint16_t *y, int32_t ldy, int32_t offy,
                  int32_t nz, int32_t ny, int32_t nx, int32_t c, void *stream);
int unet_pool_bwd(const uint16_t *dy, int32_t ldy, int32_t offy, uint16_t *dx, int32_t ldx, int32_t offx,
                  int32_t nz, int32_t ny, int32_t nx, int32_t c, void *stream);

/* Nearest-neighbour 2x upsampling from (nz/2, ny/2, nx/2) to (nz, ny, nx);
 * backward sums the eight children (overwrites dx). */
int unet_up_fwd(const uint16_t *x, int32_t ldx, int32_t offx, uint16_t *y, int32_t ldy, int32_t offy,
                int32_t nz, int32_t ny, int32_t nx, int32_t c, void *stream);
int unet_up_bwd(const uint16_t *dy, int32_t ldy, int32_t offy, uint16_t *dx, int32_t ldx, int32_t offx,
                int32_t nz, int32_t ny, int32_t nx, int32_t c, void *stream);

/* Output head (1x1x1, c -> 1, FP32): out[v] = base[v] + b + sum_c w[c] x[v, c]. */
int unet_head_fwd(const uint16_t *x, int32_t ldx, const float *w, const float *b, const float *base, float *out,
                  int64_t nvox, int32_t c, void *stream);
/* Head backward from dout (FP32): dx[v, c] = dout[v] w[c] (BF16), dw[c] += sum
 * dout[v] x[v, c], db += sum dout[v].  c <= 32. */
int unet_head_bwd(const uint16_t *x, int32_t ldx, const float *w, const float *dout, uint16_t *dx, float *dw,
                  float *db, int64_t nvox, int32_t c, void *stream);

/* Weighted masked mean squared error over voxels with mask != 0:
 * loss[0] += sum_v w[v] (pred - target)^2 / count and dout[v] = 2 w[v] (pred - target) / count,
 * with w = weight[v], or 1 when weight is NULL. */
int unet_mse(const float *pred, const float *target, const uint8_t *mask, const float *weight, float *dout,
             float *loss, int64_t nvox, int64_t count, void *stream);

/* Adam step on FP32 master weights p with moments m, v; also writes the BF16
 * copy pb (may be NULL).  t is the 1-based step number. */
int unet_adam(float *p, float *m, float *v, const float *g, uint16_t *pb, int64_t n, float lr, float beta1,
              float beta2, float eps, int32_t t, void *stream);

/* FP32 -> BF16 (round to nearest even) and zero fill helpers. */
int unet_to_bf16(const float *src, uint16_t *dst, int64_t n, void *stream);
int unet_zero(void *dst, int64_t bytes, void *stream);

/* Input features of the network (16 channels, BF16) from the solver's dense
 * fields on the simulated grid: c0 active, c1 log10(D / D_ref)/3 on active voxels
 * (D / D_ref = (tau - 1/2) / (tau_ref - 1/2), Eq. 24), c2 n_cat/6, c3 exp(-x/24),
 * c4 exp(-x/96), c5 exp(-(nx-1-x)/24) (distances from the inlet and outlet faces in
 * voxels), rest 0.  omega is 1/tau as stored by lbm_get_host_fields (uploaded to the
 * device).  When weight is not NULL it receives the training weight of each voxel:
 * min(weight_cap, (D_ref / D)^weight_power) on active voxels, 0 elsewhere (slowly
 * relaxing, low-diffusivity voxels weigh more; weight_cap >= 1, 0 <= weight_power <= 4).
 * n_cat may be NULL (c2 = 0: the effective-property problems have no sink). */
int unet_features(const uint8_t *active, const uint8_t *n_cat, const float *omega, float tau_ref,
                  uint16_t *feat, float *weight, float weight_power, float weight_cap, int32_t nz, int32_t ny,
                  int32_t nx, void *stream);

/* Log-space training target and its inverse (elementwise, in place allowed):
 * inverse == 0: dst = ln(max(src, 0) + eps); inverse != 0: dst = min(cmax, max(0,
 * exp(src) - eps)).  Training on ln(C + eps) makes the network's error relative to
 * C, which is what decides whether a start beats C = 0 in voxels where C is small.
 * eps > 0, cmax > 0. */
int unet_log_map(const float *src, float *dst, int64_t n, float eps, int32_t inverse, float cmax, void *stream);

/* Start field of the solver from a log-space prediction y (FP32, n voxels):
 * c[v] = min(cmax, max(0, exp(y[v]) - eps)) where depth[v] <= depth_max, else 0
 * (the cold-start value).  depth is the pore-depth map of lbm_get_pore_depth,
 * uploaded to the device.  Voxels deep in ionomer relax slowly and hold small
 * concentrations, so C = 0 is the better start there. */
int unet_start_field(const float *y, const uint8_t *depth, int32_t depth_max, float eps, float cmax, float *c,
                     int64_t n, void *stream);

/* Corrector target of the effective-diffusivity problem (Dirichlet c_in at the
 * face x = -1/2, c_out at x = nx - 1/2; Section 3.5.1, Eq. 19), elementwise over a dense
 * grid with x fastest (nvox a multiple of nx).  With lin(x) = c_in + (c_out - c_in)
 * (x + 1/2) / nx and s = nx / (c_in - c_out):
 *   inverse == 0: dst = s (src - lin(x));  inverse != 0: dst = min(cmax, max(0, lin(x) + src / s)).
 * The corrector of a statistically uniform structure depends on the local structure
 * only, not on the domain length, so a network trained on short domains predicts it
 * on long ones.  c_in != c_out, cmax > 0. */
int unet_corrector_map(const float *src, float *dst, int64_t nvox, int32_t nx, float c_in, float c_out,
                       int32_t inverse, float cmax, void *stream);

/* ---- The network as one object
 *
 * The fixed architecture above (four levels of 16, 32, 64 and 128 channels, two
 * 3x3x3 convolutions with ReLU per level, 2x2x2 average pooling, nearest 2x
 * upsampling with skip concatenation, 1x1x1 FP32 head; 16 input channels from
 * unet_features) on one grid nz x ny x nx (each a multiple of 8).
 *
 * Parameters are one flat FP32 array of unet_param_count() values: tensor t
 * (0..13 the convolutions in forward order e1a e1b e2a e2b e3a e3b b4a b4b d3a d3b
 * d2a d2b d1a d1b, 14 the head) has its weights at w_offset (w_count values:
 * [cout][unet_kpad(cin)] as in unet_conv3d_fwd, or the head's 16 channel weights)
 * and its bias at b_offset (cout values; the head has one).  Entries between
 * tensors are padding (zero).
 *
 * unet_create: a handle for the grid; train != 0 adds the gradient buffers and the
 *   Adam moments.  -1 for sizes that are not positive multiples of 8 or above 2^31
 *   voxels.  No device call.
 * unet_workspace_bytes / unet_bind: the caller-owned device workspace (>= the
 *   size, 256-byte aligned; parameters, their BF16 copies, activations, and when
 *   training their gradients and the moments) and the HIP stream every call
 *   enqueues on.  bind zeroes the workspace and forgets the parameters.
 * unet_set_params: copies params_dev (device, unet_param_count() FP32 values) in
 *   and makes the BF16 copies; the Adam moments and step count stay (bind zeroes
 *   them).
 * unet_get_params: copies the FP32 parameters and/or (training) the gradients of
 *   the last unet_backward out to device arrays of the same layout (either may be
 *   NULL, not both).
 * unet_forward: out_dev[v] (FP32, nz ny nx values; NULL: the internal output buffer)
 *   = network(feat_dev) + base_dev[v] (base_dev may be NULL).  feat_dev: BF16
 *   [v][16] as from unet_features (NULL: the internal feature buffer that
 *   unet_features_buffer exposes).
 * unet_backward: after unet_forward on a training handle, the gradients of the
 *   parameters for the output gradient dout_dev (FP32 per voxel), overwriting the
 *   previous ones.
 * unet_adam_step: one Adam step (bias-corrected, step count kept by the handle)
 *   of every parameter with the gradients of the last backward.
 * unet_train_step: forward, the weighted masked MSE of unet_mse against
 *   target_dev (mask_dev != 0 voxels, count of them, weight_dev may be NULL),
 *   backward and an Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with rate lr;
 *   loss_dev (may be NULL) receives the loss before the step.
 * unet_predict: the solver's start field c_dev (FP32, nz ny nx) for a structure
 *   given by the solver's dense device fields (active, n_cat (may be NULL), omega
 *   = 1/tau, as lbm_get_host_fields gives them) and tau_ref: features, forward,
 *   then the inverse of the training target per *tgt:
 *     UNET_TARGET_LOG: min(cmax, max(0, exp(y) - eps)), and 0 (the cold start)
 *       where depth (device, may be NULL) exceeds depth_max;
 *     UNET_TARGET_CORRECTOR: min(cmax, max(0, lin(x) + y (c_in - c_out) / nx))
 *       with lin the linear profile between the Dirichlet faces (Eq. 19);
 *     UNET_TARGET_PLAIN: y itself.
 * unet_features_buffer: device addresses of the handle's feature (BF16 [v][16])
 *   and output (FP32 [v]) buffers.
 * Every call returns 0, -1 for invalid arguments (NULL handle, unbound handle,
 * parameters not set, backward without a training forward before it), -6 when a
 * launch or copy failed.  One handle per thread. */
typedef struct unet_net unet_net;

enum { UNET_TARGET_LOG = 0, UNET_TARGET_CORRECTOR = 1, UNET_TARGET_PLAIN = 2 };

typedef struct {
    uint32_t struct_size;   /* = sizeof(unet_target)                               */
    int32_t kind;           /* UNET_TARGET_*                                       */
    float eps;              /* LOG: the offset of ln(C + eps)                      */
    float cmax;             /* upper clip of the start field                       */
    float c_in, c_out;      /* CORRECTOR: Dirichlet values at x = 0 and x = L      */
    const uint8_t *depth;   /* LOG: pore-depth map (lbm_get_pore_depth), or NULL   */
    int32_t depth_max;      /* LOG: keep the prediction up to this depth           */
} unet_target;

int64_t unet_param_count(void);
int unet_param_tensor(int32_t tensor, int32_t *cin, int32_t *cout, int64_t *w_offset, int64_t *w_count,
                      int64_t *b_offset);
int unet_create(int32_t nz, int32_t ny, int32_t nx, int32_t train, unet_net **out);
int unet_workspace_bytes(const unet_net *n, size_t *bytes);
int unet_bind(unet_net *n, void *workspace_dev, size_t bytes, void *stream);
int unet_set_params(unet_net *n, const float *params_dev);
int unet_get_params(const unet_net *n, float *params_dev, float *grads_dev);
int unet_forward(unet_net *n, const uint16_t *feat_dev, const float *base_dev, float *out_dev);
int unet_backward(unet_net *n, const uint16_t *feat_dev, const float *dout_dev);
int unet_adam_step(unet_net *n, float lr, float beta1, float beta2, float eps);
int unet_train_step(unet_net *n, const uint16_t *feat_dev, const float *target_dev, const uint8_t *mask_dev,
                    const float *weight_dev, int64_t count, float lr, float *loss_dev);
int unet_predict(unet_net *n, const uint8_t *active_dev, const uint8_t *n_cat_dev, const float *omega_dev,
                 float tau_ref, const unet_target *tgt, float *c_dev);
int unet_features_buffer(const unet_net *n, uint16_t **feat_dev, float **out_dev);
void unet_destroy(unet_net *n);

/* Lane-layout self check of the MFMA builtin: a = A (16x32, row major FP32),
 * b = B (32x16); writes D = A B through the kernels' fragment mapping into d
 * (16x16).  Used by the tests to pin the mapping on the device. */
int unet_mfma_selftest(const float *a, const float *b, float *d, void *stream);

#ifdef __cplusplus
}
#endif
#endif
