// Internal declarations of the learned warm start: a residual convolutional
// network that maps (log K, normalised FMG residual) on a QoI stage grid to a
// correction of the FMG start. Training kernels (FP32, planar [b][c][y][x])
// live in cnn_train.hip, BF16 inference kernels (matrix cores, activations
// [b][y][x][c]) in cnn_infer.hip, the host object and its C ABI in cnn.cpp.
#pragma once
#include "common.h"

namespace fmgmc {

constexpr int kCnnIn = 2;      // input channels: log K, r / rms(r)
constexpr int kCnnWidth = 32;  // hidden channels
constexpr int kCnnRes = 4;     // residual layers
constexpr int kCnnLayers = kCnnRes + 2;

// flat parameter layout: layer 0 (kCnnIn -> F), layers 1..R (F -> F), output (F -> 1);
// each layer W[co][ci][3][3] then b[co]
inline int cnn_layer_ci(int l) { return l == 0 ? kCnnIn : kCnnWidth; }
inline int cnn_layer_co(int l) { return l == kCnnLayers - 1 ? 1 : kCnnWidth; }
inline int64_t cnn_layer_np(int l) { return int64_t(cnn_layer_co(l)) * cnn_layer_ci(l) * 9 + cnn_layer_co(l); }
inline int64_t cnn_layer_off(int l) {
    int64_t o = 0;
    for (int k = 0; k < l; ++k) o += cnn_layer_np(k);
    return o;
}
inline int64_t cnn_nparams() { return cnn_layer_off(kCnnLayers); }

// ------------------------------------------------------------ training (FP32)
enum { CONV_FIRST = 0, CONV_RES = 1, CONV_OUT = 2, CONV_BWD = 3 };

struct ConvArgs {
    int n, B;
    const float *in;      // [B][CI][n][n]
    const float *W;       // [CO][CI][3][3] (cross-correlation weights)
    const float *bias;    // [CO] (forward modes)
    float *out;           // forward: z [B][CO][n][n]; BWD: gradient of the layer input
    float *out2;          // forward FIRST/RES: h; BWD: masked gradient (nullable)
    const float *addend;  // BWD: gradient flowing through the identity path (nullable)
    const float *mask;    // BWD: pre-activation whose sign gates out2 (nullable)
};
int launch_conv_f32(int ci, int co, int mode, const ConvArgs &a, hipStream_t st);

// Weight/bias gradients of one layer: sum over all cells of g[co] x a[ci] at
// each tap; partial sums per workgroup, then a fixed-order reduction.
struct WgradArgs {
    int n, B;
    const float *g;       // [B][CO][n][n]
    const float *a;       // [B][CI][n][n]
    float *part;          // [P][CO*CI*9 + CO]
    int P;
};
int launch_wgrad_f32(int ci, int co, const WgradArgs &a, hipStream_t st);
int launch_sum_parts(const float *part, int P, int64_t np, float *out, hipStream_t st);
// transposed weights for the data gradient: Wt[ci][co][8 - tap] = W[co][ci][tap]
int launch_flip_weights(const float *W, int ci, int co, float *Wt, hipStream_t st);
// loss (1/N) sum (y - t)^2 and dy = 2 (y - t) / N; part: [>= 1024] doubles
int launch_mse(const float *y, const float *t, int64_t N, float *dy, double *part, double *loss, hipStream_t st);
// residual loss (1/N) sum (x1 - A y)^2 with A from K = exp(x0); u = x1 - A y; dy = -2 A u / N
int launch_resid_loss(int n, int B, const float *x, const float *y, float *u, float *dy, double *part,
                      double *loss, hipStream_t st);
int launch_adam(float *theta, const float *g, float *m, float *v, int64_t np, double lr, double b1, double b2,
                double eps, int step, hipStream_t st);

// --------------------------------------------------- training-pair packing
// x[s][0] = log K, x[s][1] = r / rms(r), rms = sqrt(rr / n^2)
int launch_pack_x(int n, int S, const float *K, const float *r, const double *rr, float *x, hipStream_t st);
// t[s] = (p - p0) / rms
int launch_pack_t(int n, int S, const double *p, const double *p0, const double *rr, float *t, hipStream_t st);
// after a warm start: active[s] = (rr_new < rr_old) ? 0 : 1 (1 = restore the plain start), flag bit 2
int launch_judge(int S, const double *rr_new, const double *rr_old, int32_t *restore, uint8_t *flags,
                 hipStream_t st);
int launch_copy_f64(const double *src, double *dst, int64_t n, hipStream_t st);

// ---------------------------------------------------------- inference (BF16)
// Packed weights: per layer, MFMA B fragments in lane order (bf16) and FP32 biases.
struct CnnPacked {
    const void *w[kCnnLayers];   // bf16 fragments
    const float *b[kCnnLayers];
};
int cnn_packed_bytes(int layer);  // bytes of layer's fragments
int launch_pack_weights(const float *theta, void *const *wfrag, float *const *bias, hipStream_t st);

struct InferArgs {
    int n, S;
    // input: channel 0 = in0 (log applied if log0), channel 1 = in1 * scale1
    const float *in0;
    const float *in1;
    int64_t in_stride;    // sample stride of in0 / in1 in floats
    int log0;
    const double *rr;     // nullable: scale1 = 1 / sqrt(rr[s] / n^2), also the output scale
    // output: y (nullable) [S][n][n] = network output; or p += scale * output
    // (launch_cnn_infer); or e = scale * output in FP32 (launch_cnn_fused)
    float *y;
    double *p;
    float *e;
    const int32_t *active;  // nullable
};
// runs all layers over S samples in sub-batches; act0/act1 hold sub_batch
// samples of [n][n][32] bf16 each
int launch_cnn_infer(const InferArgs &a, const CnnPacked &w, void *act0, void *act1, int sub_batch,
                     hipStream_t st);
// all layers in one pass, activations on chip (same results as launch_cnn_infer)
int launch_cnn_fused(const InferArgs &a, const CnnPacked &w, hipStream_t st);

}  // namespace fmgmc

// The network object behind the C ABI (device-resident parameters, Adam
// moments, packed inference weights and a training workspace).
struct fmgmc_cnn {
    int device = 0;
    float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;  // [NP]
    int64_t step = 0;
    void *wfrag[fmgmc::kCnnLayers] = {};
    float *bias[fmgmc::kCnnLayers] = {};
    bool packed = false;  // inference fragments match theta
    // training workspace, sized for cap_cells = batch * n * n
    int64_t cap_cells = 0;
    float *z[fmgmc::kCnnLayers - 1] = {}, *h[fmgmc::kCnnLayers - 1] = {};
    float *y = nullptr, *dy = nullptr, *dh[2] = {}, *dz[2] = {}, *wt = nullptr, *part = nullptr;
    double *mse_part = nullptr, *loss = nullptr;
    // inference workspace for fmgmc_cnn_forward (BF16)
    int64_t cap_act = 0;
    void *act[2] = {};
};

namespace fmgmc {
// packs the inference fragments if theta changed (stream-ordered)
int cnn_ensure_packed(fmgmc_cnn *c, hipStream_t st);
CnnPacked cnn_packed(const fmgmc_cnn *c);
// training-pair workspace views of a solve (set by fmgmc_cnn_make_data)
int cnn_grad_impl(fmgmc_cnn *c, int n, int B, const float *x, const float *t, int kind, double *loss,
                  hipStream_t st);
int cnn_adam_impl(fmgmc_cnn *c, double lr, hipStream_t st);
}  // namespace fmgmc
