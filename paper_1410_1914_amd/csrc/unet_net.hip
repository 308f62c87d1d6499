// The warm-start network as one object behind the C ABI (include/unet.h): a 3-D
// U-Net of four levels (16, 32, 64, 128 channels) on a fixed grid, its parameters in
// one flat FP32 array with a BF16 mirror, the activation buffers of the forward
// pass, and (for training) their gradients, the parameter gradients and the Adam
// moments.  Every operation is a launch of the layer kernels of unet_kernels.hip on
// the bound stream; the object only lays out memory and orders the launches.
//
// Forward: two 3x3x3 convolutions with ReLU per level, 2x2x2 average pooling down,
// nearest 2x upsampling and channel concatenation with the skip tensor up, and a
// 1x1x1 FP32 head.  Backward: the adjoint of every step in reverse order (ReLU
// mask, weight gradient on MFMA, backward data as a forward convolution with the
// flipped, transposed weights).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <new>

#include "include/unet.h"

namespace {

constexpr int kIn = 16;
constexpr int kC1 = 16, kC2 = 32, kC3 = 64, kC4 = 128;
constexpr int kLayers = 14;  // 3x3x3 convolutions; the head is parameter tensor 14

struct LayerSpec {
    int cin, cout;
};
// forward order: e1a e1b e2a e2b e3a e3b b4a b4b d3a d3b d2a d2b d1a d1b
constexpr LayerSpec kSpec[kLayers] = {{kIn, kC1}, {kC1, kC1}, {kC1, kC2}, {kC2, kC2}, {kC2, kC3},
                                      {kC3, kC3}, {kC3, kC4}, {kC4, kC4}, {kC4 + kC3, kC3}, {kC3, kC3},
                                      {kC3 + kC2, kC2}, {kC2, kC2}, {kC2 + kC1, kC1}, {kC1, kC1}};
enum { E1A, E1B, E2A, E2B, E3A, E3B, B4A, B4B, D3A, D3B, D2A, D2B, D1A, D1B };

constexpr int64_t align64(int64_t n) { return (n + 63) / 64 * 64; }

struct ParamLayout {
    int64_t w[kLayers + 1], b[kLayers + 1], wlen[kLayers + 1];
    int64_t total;
};

ParamLayout param_layout() {
    ParamLayout L{};
    int64_t o = 0;
    for (int l = 0; l <= kLayers; ++l) {
        const int64_t wl = l < kLayers ? (int64_t)kSpec[l].cout * unet_kpad(kSpec[l].cin) : kC1;
        const int64_t bl = l < kLayers ? kSpec[l].cout : 1;
        L.w[l] = o;
        L.wlen[l] = wl;
        o = align64(o + wl);
        L.b[l] = o;
        o = align64(o + bl);
    }
    L.total = o;
    return L;
}

// activation buffers, BF16 with the channel count as the row stride
enum Act { A_FEAT, A_A1, A_CAT1, A_D1A, A_D1B, A_P2, A_A2, A_CAT2, A_D2A, A_D2B, A_P3, A_A3, A_CAT3, A_D3A, A_D3B,
           A_P4, A_B4A, A_B4B, A_COUNT };
constexpr int kActLevel[A_COUNT] = {0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 3, 3, 3};
constexpr int kActCh[A_COUNT] = {kIn, kC1, kC1 + kC2, kC1, kC1, kC1, kC2, kC2 + kC3, kC2, kC2,
                                 kC2, kC3, kC3 + kC4, kC3, kC3, kC3, kC4, kC4};

hipError_t to_hip(int st) { return st == 0 ? hipSuccess : (st == -1 ? hipErrorInvalidValue : hipErrorLaunchFailure); }

}  // namespace

struct unet_net {
    int nz, ny, nx, train;
    int dims[4][3];
    int64_t vox[4];
    ParamLayout P;
    size_t off_p, off_pb, off_g, off_m, off_v, off_act[A_COUNT], off_out, off_gact[A_COUNT], off_gout, off_wt,
        off_loss, bytes;
    char *ws = nullptr;
    hipStream_t st = nullptr;
    int32_t t = 0;  // Adam steps taken
    bool have_params = false, forward_train = false;

    template <class T>
    T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
    float *p() const { return at<float>(off_p); }
    uint16_t *pb() const { return at<uint16_t>(off_pb); }
    float *g() const { return at<float>(off_g); }
    uint16_t *act(int a) const { return at<uint16_t>(off_act[a]); }
    uint16_t *gact(int a) const { return at<uint16_t>(off_gact[a]); }

    void layout() {
        P = param_layout();
        for (int l = 0; l < 4; ++l) {
            dims[l][0] = nz >> l;
            dims[l][1] = ny >> l;
            dims[l][2] = nx >> l;
            vox[l] = (int64_t)dims[l][0] * dims[l][1] * dims[l][2];
        }
        size_t o = 0;
        auto take = [&](size_t n) {
            const size_t at = o;
            o = (o + n + 255) / 256 * 256;
            return at;
        };
        off_p = take(sizeof(float) * P.total);
        off_pb = take(sizeof(uint16_t) * P.total);
        off_g = off_m = off_v = 0;
        if (train) {
            off_g = take(sizeof(float) * P.total);
            off_m = take(sizeof(float) * P.total);
            off_v = take(sizeof(float) * P.total);
        }
        for (int a = 0; a < A_COUNT; ++a) off_act[a] = take(sizeof(uint16_t) * vox[kActLevel[a]] * kActCh[a]);
        off_out = take(sizeof(float) * vox[0]);
        off_gout = off_wt = off_loss = 0;
        for (int a = 0; a < A_COUNT; ++a) off_gact[a] = 0;
        if (train) {
            for (int a = A_A1; a < A_COUNT; ++a) off_gact[a] = take(sizeof(uint16_t) * vox[kActLevel[a]] * kActCh[a]);
            off_gout = take(sizeof(float) * vox[0]);
            int64_t wt = 0;
            for (int l = 0; l < kLayers; ++l) {
                const int64_t n = (int64_t)kSpec[l].cin * unet_kpad(kSpec[l].cout);
                wt = n > wt ? n : wt;
            }
            off_wt = take(sizeof(uint16_t) * wt);
            off_loss = take(sizeof(float) * 64);
        }
        bytes = o;
    }

    // one 3x3x3 convolution of layer l on level lev: x (ldx, offx) -> y (ldy, offy)
    hipError_t conv(int l, const uint16_t *x, int ldx, int offx, uint16_t *y, int ldy, int offy, int lev, bool relu) {
        const int *d = dims[lev];
        return to_hip(unet_conv3d_fwd(x, ldx, offx, pb() + P.w[l], p() + P.b[l], y, ldy, offy, nullptr, d[0], d[1],
                                      d[2], kSpec[l].cin, kSpec[l].cout, relu ? 1 : 0, st));
    }

    // a decoder convolution of layer l on level lev over [skip x (c1 channels), the
    // level below's x2 (c2 channels) upsampled], the concatenation never stored
    hipError_t conv_cat(int l, const uint16_t *x, int c1, const uint16_t *x2, int c2, uint16_t *y, int lev) {
        const int *d = dims[lev];
        return to_hip(unet_conv3d_fwd_cat(x, c1, 0, c1, x2, c2, 0, pb() + P.w[l], p() + P.b[l], y, kSpec[l].cout, 0,
                                          nullptr, d[0], d[1], d[2], kSpec[l].cin, kSpec[l].cout, 1, st));
    }

    hipError_t forward(const uint16_t *feat, const float *base, float *out) {
        hipError_t e = hipSuccess;
        auto run = [&](hipError_t r) {
            if (e == hipSuccess) e = r;
        };
        const int *d0 = dims[0], *d1 = dims[1], *d2 = dims[2];
        if (!train) {
            // Inference: each skip tensor stays in rows of its own channels (in the
            // front of its concatenation's buffer) and each decoder convolution reads
            // the level below upsampled in place, so no concatenation is written and
            // pooling reads whole rows.  Training keeps the concatenations: the weight
            // gradients read them.
            run(conv(E1A, feat, kIn, 0, act(A_A1), kC1, 0, 0, true));
            run(conv(E1B, act(A_A1), kC1, 0, act(A_CAT1), kC1, 0, 0, true));
            run(to_hip(unet_pool_fwd(act(A_CAT1), kC1, 0, act(A_P2), kC1, 0, d0[0], d0[1], d0[2], kC1, st)));
            run(conv(E2A, act(A_P2), kC1, 0, act(A_A2), kC2, 0, 1, true));
            run(conv(E2B, act(A_A2), kC2, 0, act(A_CAT2), kC2, 0, 1, true));
            run(to_hip(unet_pool_fwd(act(A_CAT2), kC2, 0, act(A_P3), kC2, 0, d1[0], d1[1], d1[2], kC2, st)));
            run(conv(E3A, act(A_P3), kC2, 0, act(A_A3), kC3, 0, 2, true));
            run(conv(E3B, act(A_A3), kC3, 0, act(A_CAT3), kC3, 0, 2, true));
            run(to_hip(unet_pool_fwd(act(A_CAT3), kC3, 0, act(A_P4), kC3, 0, d2[0], d2[1], d2[2], kC3, st)));
            run(conv(B4A, act(A_P4), kC3, 0, act(A_B4A), kC4, 0, 3, true));
            run(conv(B4B, act(A_B4A), kC4, 0, act(A_B4B), kC4, 0, 3, true));
            run(conv_cat(D3A, act(A_CAT3), kC3, act(A_B4B), kC4, act(A_D3A), 2));
            run(conv(D3B, act(A_D3A), kC3, 0, act(A_D3B), kC3, 0, 2, true));
            run(conv_cat(D2A, act(A_CAT2), kC2, act(A_D3B), kC3, act(A_D2A), 1));
            run(conv(D2B, act(A_D2A), kC2, 0, act(A_D2B), kC2, 0, 1, true));
            run(conv_cat(D1A, act(A_CAT1), kC1, act(A_D2B), kC2, act(A_D1A), 0));
            // the last convolution with the head in its epilogue: D1B is never stored
            static_assert(kC1 == 16, "unet_conv3d_fwd_head is the 16-channel form");
            run(to_hip(unet_conv3d_fwd_head(act(A_D1A), kC1, 0, pb() + P.w[D1B], p() + P.b[D1B], p() + P.w[kLayers],
                                            p() + P.b[kLayers], base, out, d0[0], d0[1], d0[2], st)));
            return e;
        }
        run(conv(E1A, feat, kIn, 0, act(A_A1), kC1, 0, 0, true));
        run(conv(E1B, act(A_A1), kC1, 0, act(A_CAT1), kC1 + kC2, 0, 0, true));
        run(to_hip(unet_pool_fwd(act(A_CAT1), kC1 + kC2, 0, act(A_P2), kC1, 0, d0[0], d0[1], d0[2], kC1, st)));
        run(conv(E2A, act(A_P2), kC1, 0, act(A_A2), kC2, 0, 1, true));
        run(conv(E2B, act(A_A2), kC2, 0, act(A_CAT2), kC2 + kC3, 0, 1, true));
        run(to_hip(unet_pool_fwd(act(A_CAT2), kC2 + kC3, 0, act(A_P3), kC2, 0, d1[0], d1[1], d1[2], kC2, st)));
        run(conv(E3A, act(A_P3), kC2, 0, act(A_A3), kC3, 0, 2, true));
        run(conv(E3B, act(A_A3), kC3, 0, act(A_CAT3), kC3 + kC4, 0, 2, true));
        run(to_hip(unet_pool_fwd(act(A_CAT3), kC3 + kC4, 0, act(A_P4), kC3, 0, d2[0], d2[1], d2[2], kC3, st)));
        run(conv(B4A, act(A_P4), kC3, 0, act(A_B4A), kC4, 0, 3, true));
        run(conv(B4B, act(A_B4A), kC4, 0, act(A_B4B), kC4, 0, 3, true));
        run(to_hip(unet_up_fwd(act(A_B4B), kC4, 0, act(A_CAT3), kC3 + kC4, kC3, d2[0], d2[1], d2[2], kC4, st)));
        run(conv(D3A, act(A_CAT3), kC3 + kC4, 0, act(A_D3A), kC3, 0, 2, true));
        run(conv(D3B, act(A_D3A), kC3, 0, act(A_D3B), kC3, 0, 2, true));
        run(to_hip(unet_up_fwd(act(A_D3B), kC3, 0, act(A_CAT2), kC2 + kC3, kC2, d1[0], d1[1], d1[2], kC3, st)));
        run(conv(D2A, act(A_CAT2), kC2 + kC3, 0, act(A_D2A), kC2, 0, 1, true));
        run(conv(D2B, act(A_D2A), kC2, 0, act(A_D2B), kC2, 0, 1, true));
        run(to_hip(unet_up_fwd(act(A_D2B), kC2, 0, act(A_CAT1), kC1 + kC2, kC1, d0[0], d0[1], d0[2], kC2, st)));
        run(conv(D1A, act(A_CAT1), kC1 + kC2, 0, act(A_D1A), kC1, 0, 0, true));
        run(conv(D1B, act(A_D1A), kC1, 0, act(A_D1B), kC1, 0, 0, true));
        run(to_hip(unet_head_fwd(act(A_D1B), kC1, p() + P.w[kLayers], p() + P.b[kLayers], base, out, vox[0], kC1,
                                 st)));
        return e;
    }

    // Backward of one convolution: gy holds dL/dy (after the ReLU) and becomes
    // dL/d(pre-activation); the weight and bias gradients accumulate into g();
    // dL/dx is written into gx unless gx is null.
    hipError_t conv_bwd(int l, const uint16_t *x, int ldx, int offx, const uint16_t *y, int ldy, int offy, uint16_t *gy,
                        int ldg, int offg, uint16_t *gx, int ldgx, int offgx, int lev) {
        const int *d = dims[lev];
        const int cin = kSpec[l].cin, cout = kSpec[l].cout;
        int s = unet_relu_bwd(y, ldy, offy, gy, ldg, offg, vox[lev], cout, st);
        if (s == 0)
            s = unet_conv3d_wgrad(x, ldx, offx, gy, ldg, offg, d[0], d[1], d[2], cin, cout, g() + P.w[l], g() + P.b[l],
                                  st);
        if (s == 0 && gx) {
            uint16_t *wt = at<uint16_t>(off_wt);
            s = unet_conv3d_wtrans(pb() + P.w[l], wt, cin, cout, st);
            if (s == 0)
                s = unet_conv3d_fwd(gy, ldg, offg, wt, nullptr, gx, ldgx, offgx, nullptr, d[0], d[1], d[2], cout, cin, 0,
                                    st);
        }
        return to_hip(s);
    }

    hipError_t backward(const uint16_t *feat, const float *dout) {
        hipError_t e = to_hip(unet_zero(g(), (int64_t)sizeof(float) * P.total, st));
        auto run = [&](hipError_t r) {
            if (e == hipSuccess) e = r;
        };
        for (int a : {A_CAT1, A_CAT2, A_CAT3})
            run(to_hip(unet_zero(gact(a), (int64_t)sizeof(uint16_t) * vox[kActLevel[a]] * kActCh[a], st)));
        const int *d0 = dims[0], *d1 = dims[1], *d2 = dims[2];
        run(to_hip(unet_head_bwd(act(A_D1B), kC1, p() + P.w[kLayers], dout, gact(A_D1B), g() + P.w[kLayers],
                                 g() + P.b[kLayers], vox[0], kC1, st)));
        run(conv_bwd(D1B, act(A_D1A), kC1, 0, act(A_D1B), kC1, 0, gact(A_D1B), kC1, 0, gact(A_D1A), kC1, 0, 0));
        run(conv_bwd(D1A, act(A_CAT1), kC1 + kC2, 0, act(A_D1A), kC1, 0, gact(A_D1A), kC1, 0, gact(A_CAT1), kC1 + kC2,
                     0, 0));
        run(to_hip(unet_up_bwd(gact(A_CAT1), kC1 + kC2, kC1, gact(A_D2B), kC2, 0, d0[0], d0[1], d0[2], kC2, st)));
        run(conv_bwd(D2B, act(A_D2A), kC2, 0, act(A_D2B), kC2, 0, gact(A_D2B), kC2, 0, gact(A_D2A), kC2, 0, 1));
        run(conv_bwd(D2A, act(A_CAT2), kC2 + kC3, 0, act(A_D2A), kC2, 0, gact(A_D2A), kC2, 0, gact(A_CAT2), kC2 + kC3,
                     0, 1));
        run(to_hip(unet_up_bwd(gact(A_CAT2), kC2 + kC3, kC2, gact(A_D3B), kC3, 0, d1[0], d1[1], d1[2], kC3, st)));
        run(conv_bwd(D3B, act(A_D3A), kC3, 0, act(A_D3B), kC3, 0, gact(A_D3B), kC3, 0, gact(A_D3A), kC3, 0, 2));
        run(conv_bwd(D3A, act(A_CAT3), kC3 + kC4, 0, act(A_D3A), kC3, 0, gact(A_D3A), kC3, 0, gact(A_CAT3), kC3 + kC4,
                     0, 2));
        run(to_hip(unet_up_bwd(gact(A_CAT3), kC3 + kC4, kC3, gact(A_B4B), kC4, 0, d2[0], d2[1], d2[2], kC4, st)));
        run(conv_bwd(B4B, act(A_B4A), kC4, 0, act(A_B4B), kC4, 0, gact(A_B4B), kC4, 0, gact(A_B4A), kC4, 0, 3));
        run(conv_bwd(B4A, act(A_P4), kC3, 0, act(A_B4A), kC4, 0, gact(A_B4A), kC4, 0, gact(A_P4), kC3, 0, 3));
        run(to_hip(unet_pool_bwd(gact(A_P4), kC3, 0, gact(A_CAT3), kC3 + kC4, 0, d2[0], d2[1], d2[2], kC3, st)));
        run(conv_bwd(E3B, act(A_A3), kC3, 0, act(A_CAT3), kC3 + kC4, 0, gact(A_CAT3), kC3 + kC4, 0, gact(A_A3), kC3, 0,
                     2));
        run(conv_bwd(E3A, act(A_P3), kC2, 0, act(A_A3), kC3, 0, gact(A_A3), kC3, 0, gact(A_P3), kC2, 0, 2));
        run(to_hip(unet_pool_bwd(gact(A_P3), kC2, 0, gact(A_CAT2), kC2 + kC3, 0, d1[0], d1[1], d1[2], kC2, st)));
        run(conv_bwd(E2B, act(A_A2), kC2, 0, act(A_CAT2), kC2 + kC3, 0, gact(A_CAT2), kC2 + kC3, 0, gact(A_A2), kC2, 0,
                     1));
        run(conv_bwd(E2A, act(A_P2), kC1, 0, act(A_A2), kC2, 0, gact(A_A2), kC2, 0, gact(A_P2), kC1, 0, 1));
        run(to_hip(unet_pool_bwd(gact(A_P2), kC1, 0, gact(A_CAT1), kC1 + kC2, 0, d0[0], d0[1], d0[2], kC1, st)));
        run(conv_bwd(E1B, act(A_A1), kC1, 0, act(A_CAT1), kC1 + kC2, 0, gact(A_CAT1), kC1 + kC2, 0, gact(A_A1), kC1, 0,
                     0));
        run(conv_bwd(E1A, feat, kIn, 0, act(A_A1), kC1, 0, gact(A_A1), kC1, 0, nullptr, 0, 0, 0));
        return e;
    }
};

namespace {

int ok_net(const unet_net *n) { return n && n->ws ? 0 : -1; }

int status_of(hipError_t e) { return e == hipSuccess ? 0 : (e == hipErrorInvalidValue ? -1 : -6); }

}  // namespace

extern "C" {

int64_t unet_param_count(void) { return param_layout().total; }

int unet_param_tensor(int32_t tensor, int32_t *cin, int32_t *cout, int64_t *w_offset, int64_t *w_count,
                      int64_t *b_offset) {
    if (tensor < 0 || tensor > kLayers) return -1;
    const ParamLayout L = param_layout();
    if (cin) *cin = tensor < kLayers ? kSpec[tensor].cin : kC1;
    if (cout) *cout = tensor < kLayers ? kSpec[tensor].cout : 1;
    if (w_offset) *w_offset = L.w[tensor];
    if (w_count) *w_count = L.wlen[tensor];
    if (b_offset) *b_offset = L.b[tensor];
    return 0;
}

int unet_create(int32_t nz, int32_t ny, int32_t nx, int32_t train, unet_net **out) {
    if (!out) return -1;
    *out = nullptr;
    if (nz < 8 || ny < 8 || nx < 8 || nz % 8 || ny % 8 || nx % 8) return -1;
    if ((int64_t)nz * ny * nx > (int64_t)1 << 31) return -1;
    unet_net *n = new (std::nothrow) unet_net();
    if (!n) return -1;
    n->nz = nz;
    n->ny = ny;
    n->nx = nx;
    n->train = train ? 1 : 0;
    n->layout();
    *out = n;
    return 0;
}

int unet_workspace_bytes(const unet_net *n, size_t *bytes) {
    if (!n || !bytes) return -1;
    *bytes = n->bytes;
    return 0;
}

int unet_bind(unet_net *n, void *workspace_dev, size_t bytes, void *stream) {
    if (!n || !workspace_dev || bytes < n->bytes || (reinterpret_cast<uintptr_t>(workspace_dev) & 255)) return -1;
    n->ws = static_cast<char *>(workspace_dev);
    n->st = static_cast<hipStream_t>(stream);
    n->have_params = false;
    n->forward_train = false;
    n->t = 0;
    int s = unet_zero(n->ws, (int64_t)n->bytes, n->st);
    return s;
}

int unet_set_params(unet_net *n, const float *params_dev) {
    if (ok_net(n) || !params_dev) return -1;
    const int64_t P = n->P.total;
    hipError_t e = hipMemcpyAsync(n->p(), params_dev, sizeof(float) * P, hipMemcpyDeviceToDevice, n->st);
    if (e != hipSuccess) return -6;
    const int s = unet_to_bf16(n->p(), n->pb(), P, n->st);
    if (s == 0) n->have_params = true;
    return s;
}

int unet_get_params(const unet_net *n, float *params_dev, float *grads_dev) {
    if (ok_net(n) || (!params_dev && !grads_dev) || (grads_dev && !n->train)) return -1;
    const size_t b = sizeof(float) * n->P.total;
    hipError_t e = hipSuccess;
    if (params_dev) e = hipMemcpyAsync(params_dev, n->p(), b, hipMemcpyDeviceToDevice, n->st);
    if (e == hipSuccess && grads_dev) e = hipMemcpyAsync(grads_dev, n->g(), b, hipMemcpyDeviceToDevice, n->st);
    return e == hipSuccess ? 0 : -6;
}

int unet_forward(unet_net *n, const uint16_t *feat_dev, const float *base_dev, float *out_dev) {
    if (ok_net(n) || !n->have_params) return -1;
    const uint16_t *feat = feat_dev ? feat_dev : n->act(A_FEAT);
    float *out = out_dev ? out_dev : n->at<float>(n->off_out);
    const int s = status_of(n->forward(feat, base_dev, out));
    n->forward_train = s == 0 && n->train;
    return s;
}

int unet_backward(unet_net *n, const uint16_t *feat_dev, const float *dout_dev) {
    if (ok_net(n) || !n->train || !n->forward_train || !dout_dev) return -1;
    const uint16_t *feat = feat_dev ? feat_dev : n->act(A_FEAT);
    return status_of(n->backward(feat, dout_dev));
}

int unet_adam_step(unet_net *n, float lr, float beta1, float beta2, float eps) {
    if (ok_net(n) || !n->train || !n->have_params || !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
        !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return -1;
    n->t += 1;
    // one step over the whole flat array; the BF16 mirror follows (bias entries of the
    // mirror are never read)
    return unet_adam(n->p(), n->at<float>(n->off_m), n->at<float>(n->off_v), n->g(), n->pb(), n->P.total, lr, beta1,
                     beta2, eps, n->t, n->st);
}

int unet_train_step(unet_net *n, const uint16_t *feat_dev, const float *target_dev, const uint8_t *mask_dev,
                    const float *weight_dev, int64_t count, float lr, float *loss_dev) {
    if (ok_net(n) || !n->train || !target_dev || !mask_dev || count <= 0) return -1;
    float *out = n->at<float>(n->off_out);
    float *gout = n->at<float>(n->off_gout);
    float *loss = loss_dev ? loss_dev : n->at<float>(n->off_loss);
    int s = unet_forward(n, feat_dev, nullptr, out);
    if (s == 0) s = unet_zero(loss, sizeof(float), n->st);
    if (s == 0) s = unet_mse(out, target_dev, mask_dev, weight_dev, gout, loss, n->vox[0], count, n->st);
    if (s == 0) s = unet_backward(n, feat_dev, gout);
    if (s == 0) s = unet_adam_step(n, lr, 0.9f, 0.999f, 1e-8f);
    return s;
}

int unet_predict(unet_net *n, const uint8_t *active_dev, const uint8_t *n_cat_dev, const float *omega_dev,
                 float tau_ref, const unet_target *tgt, float *c_dev) {
    if (ok_net(n) || !n->have_params || !active_dev || !omega_dev || !tgt || !c_dev) return -1;
    if (tgt->struct_size != sizeof(unet_target)) return -1;
    int s = unet_features(active_dev, n_cat_dev, omega_dev, tau_ref, n->act(A_FEAT), nullptr, 0.f, 1.f, n->nz, n->ny,
                          n->nx, n->st);
    float *out = n->at<float>(n->off_out);
    if (s == 0) s = status_of(n->forward(n->act(A_FEAT), nullptr, out));
    n->forward_train = false;
    if (s != 0) return s;
    const int64_t V = n->vox[0];
    switch (tgt->kind) {
        case UNET_TARGET_LOG:
            if (tgt->depth)
                return unet_start_field(out, tgt->depth, tgt->depth_max, tgt->eps, tgt->cmax, c_dev, V, n->st);
            return unet_log_map(out, c_dev, V, tgt->eps, 1, tgt->cmax, n->st);
        case UNET_TARGET_CORRECTOR:
            return unet_corrector_map(out, c_dev, V, n->nx, tgt->c_in, tgt->c_out, 1, tgt->cmax, n->st);
        case UNET_TARGET_PLAIN:
            return hipMemcpyAsync(c_dev, out, sizeof(float) * V, hipMemcpyDeviceToDevice, n->st) == hipSuccess ? 0 : -6;
        default:
            return -1;
    }
}

int unet_features_buffer(const unet_net *n, uint16_t **feat_dev, float **out_dev) {
    if (ok_net(n)) return -1;
    if (feat_dev) *feat_dev = n->act(A_FEAT);
    if (out_dev) *out_dev = n->at<float>(n->off_out);
    return 0;
}

void unet_destroy(unet_net *n) { delete n; }

}  // extern "C"
