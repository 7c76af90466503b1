// Host side of the warm-start network: parameters, initialisation, file
// format, the FP32 training step (forward, loss, backward, Adam) and the BF16
// forward used by tests. Solver integration (training pairs from the FMG pass,
// warm start of a QoI stage) lives in api.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>

#include "cnn.h"

using namespace fmgmc;

namespace {

template <typename T>
int dalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) return FMGMC_OK;
    if (hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc failed (" + std::to_string(count * sizeof(T)) + " bytes)");
        return FMGMC_ENOMEM;
    }
    return FMGMC_OK;
}

template <typename T>
void dfree(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

#define TRY(x)                           \
    do {                                 \
        int rc_ = (x);                   \
        if (rc_ != FMGMC_OK) return rc_; \
    } while (0)

struct DevGuard {
    int prev = -1;
    explicit DevGuard(int d) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        (void)hipSetDevice(d);
    }
    ~DevGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// splitmix64 and Box-Muller: a deterministic normal stream for initialisation
struct Rng {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return (double(next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
    double normal() {
        const double u = uniform(), v = uniform();
        return std::sqrt(-2.0 * std::log(u)) * std::cos(6.283185307179586 * v);
    }
};

void free_train(fmgmc_cnn *c) {
    for (int l = 0; l < kCnnLayers - 1; ++l) {
        dfree(c->z[l]);
        dfree(c->h[l]);
    }
    dfree(c->y);
    dfree(c->dy);
    for (int k = 0; k < 2; ++k) {
        dfree(c->dh[k]);
        dfree(c->dz[k]);
    }
    dfree(c->wt);
    dfree(c->part);
    dfree(c->mse_part);
    dfree(c->loss);
    c->cap_cells = 0;
}

constexpr int kMaxParts = 1024;

int ensure_train(fmgmc_cnn *c, int64_t cells) {
    if (cells <= c->cap_cells) return FMGMC_OK;
    free_train(c);
    const size_t F = kCnnWidth;
    for (int l = 0; l < kCnnLayers - 1; ++l) {
        TRY(dalloc(&c->z[l], F * cells));
        TRY(dalloc(&c->h[l], F * cells));
    }
    TRY(dalloc(&c->y, size_t(cells)));
    TRY(dalloc(&c->dy, size_t(cells)));
    for (int k = 0; k < 2; ++k) {
        TRY(dalloc(&c->dh[k], F * cells));
        TRY(dalloc(&c->dz[k], F * cells));
    }
    TRY(dalloc(&c->wt, size_t(kCnnWidth) * kCnnWidth * 9));
    TRY(dalloc(&c->part, size_t(kMaxParts) * cnn_layer_np(1)));
    TRY(dalloc(&c->mse_part, 1024));
    TRY(dalloc(&c->loss, 1));
    c->cap_cells = cells;
    return FMGMC_OK;
}

int check_shape(int n, int64_t B) {
    if (n < 16 || n > 1024 || (n & (n - 1)) || B < 1 || B > 65535) {
        set_error("cnn: n must be a power of two in [16, 1024] and 1 <= batch <= 65535");
        return FMGMC_EINVAL;
    }
    return FMGMC_OK;
}

bool is_dev(const void *p) {
    hipPointerAttribute_t at;
    if (!p || hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

// FP32 forward of B samples into c->z, c->h, c->y
int forward_f32(fmgmc_cnn *c, int n, int B, const float *x, hipStream_t st) {
    ConvArgs a{};
    a.n = n;
    a.B = B;
    a.in = x;
    a.W = c->theta + cnn_layer_off(0);
    a.bias = a.W + size_t(kCnnWidth) * kCnnIn * 9;
    a.out = c->z[0];
    a.out2 = c->h[0];
    TRY(launch_conv_f32(kCnnIn, kCnnWidth, CONV_FIRST, a, st));
    for (int l = 1; l <= kCnnRes; ++l) {
        a.in = c->h[l - 1];
        a.W = c->theta + cnn_layer_off(l);
        a.bias = a.W + size_t(kCnnWidth) * kCnnWidth * 9;
        a.out = c->z[l];
        a.out2 = c->h[l];
        TRY(launch_conv_f32(kCnnWidth, kCnnWidth, CONV_RES, a, st));
    }
    a.in = c->h[kCnnRes];
    a.W = c->theta + cnn_layer_off(kCnnLayers - 1);
    a.bias = a.W + kCnnWidth * 9;
    a.out = c->y;
    a.out2 = nullptr;
    return launch_conv_f32(kCnnWidth, 1, CONV_OUT, a, st);
}

int wgrad(fmgmc_cnn *c, int layer, int n, int B, const float *g, const float *act, hipStream_t st) {
    WgradArgs w{};
    w.n = n;
    w.B = B;
    w.g = g;
    w.a = act;
    w.part = c->part;
    const int64_t tiles = int64_t(B) * (n / 16) * (n / 16);
    w.P = int(std::min<int64_t>(tiles, kMaxParts));
    TRY(launch_wgrad_f32(cnn_layer_ci(layer), cnn_layer_co(layer), w, st));
    return launch_sum_parts(c->part, w.P, cnn_layer_np(layer), c->grad + cnn_layer_off(layer), st);
}

}  // namespace

namespace fmgmc {

int cnn_ensure_packed(fmgmc_cnn *c, hipStream_t st) {
    if (c->packed) return FMGMC_OK;
    TRY(launch_pack_weights(c->theta, c->wfrag, c->bias, st));
    c->packed = true;
    return FMGMC_OK;
}

CnnPacked cnn_packed(const fmgmc_cnn *c) {
    CnnPacked p{};
    for (int l = 0; l < kCnnLayers; ++l) {
        p.w[l] = c->wfrag[l];
        p.b[l] = c->bias[l];
    }
    return p;
}

int cnn_grad_impl(fmgmc_cnn *c, int n, int B, const float *x, const float *t, int kind, double *loss,
                  hipStream_t st) {
    TRY(check_shape(n, B));
    const int64_t cells = int64_t(B) * n * n;
    TRY(ensure_train(c, cells));
    TRY(forward_f32(c, n, B, x, st));
    if (kind == FMGMC_CNN_LOSS_ERROR) TRY(launch_mse(c->y, t, cells, c->dy, c->mse_part, c->loss, st));
    else TRY(launch_resid_loss(n, B, x, c->y, c->dh[1], c->dy, c->mse_part, c->loss, st));
    // output layer
    const int Lo = kCnnLayers - 1;
    TRY(wgrad(c, Lo, n, B, c->dy, c->h[kCnnRes], st));
    TRY(launch_flip_weights(c->theta + cnn_layer_off(Lo), kCnnWidth, 1, c->wt, st));
    ConvArgs a{};
    a.n = n;
    a.B = B;
    a.in = c->dy;
    a.W = c->wt;
    a.out = c->dh[0];
    a.out2 = c->dz[0];
    a.mask = c->z[kCnnRes];
    TRY(launch_conv_f32(1, kCnnWidth, CONV_BWD, a, st));
    int cur = 0;
    for (int l = kCnnRes; l >= 1; --l) {
        TRY(wgrad(c, l, n, B, c->dz[cur], c->h[l - 1], st));
        TRY(launch_flip_weights(c->theta + cnn_layer_off(l), kCnnWidth, kCnnWidth, c->wt, st));
        a.in = c->dz[cur];
        a.addend = c->dh[cur];
        a.out = c->dh[1 - cur];
        a.out2 = c->dz[1 - cur];
        a.mask = c->z[l - 1];
        TRY(launch_conv_f32(kCnnWidth, kCnnWidth, CONV_BWD, a, st));
        cur = 1 - cur;
    }
    TRY(wgrad(c, 0, n, B, c->dz[cur], x, st));
    if (loss) {
        FMGMC_HIP(hipMemcpyAsync(loss, c->loss, sizeof(double), hipMemcpyDeviceToHost, st));
        FMGMC_HIP(hipStreamSynchronize(st));
    }
    return FMGMC_OK;
}

int cnn_adam_impl(fmgmc_cnn *c, double lr, hipStream_t st) {
    ++c->step;
    c->packed = false;
    return launch_adam(c->theta, c->grad, c->m, c->v, cnn_nparams(), lr, 0.9, 0.999, 1e-8, int(c->step), st);
}

}  // namespace fmgmc

extern "C" {

int fmgmc_cnn_create(fmgmc_cnn **out, uint64_t seed, int32_t device) {
    if (!out) {
        set_error("fmgmc_cnn_create: out is NULL");
        return FMGMC_EINVAL;
    }
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        set_error("fmgmc_cnn_create: no such HIP device");
        return FMGMC_EHIP;
    }
    DevGuard g(device);
    std::unique_ptr<fmgmc_cnn> c(new fmgmc_cnn());
    c->device = device;
    const int64_t NP = cnn_nparams();
    int rc = FMGMC_OK;
    auto fail = [&](int r) {
        fmgmc_cnn *p = c.release();
        fmgmc_cnn_destroy(p);
        return r;
    };
    if ((rc = dalloc(&c->theta, NP)) || (rc = dalloc(&c->grad, NP)) || (rc = dalloc(&c->m, NP)) ||
        (rc = dalloc(&c->v, NP)))
        return fail(rc);
    for (int l = 0; l < kCnnLayers; ++l)
        if ((rc = dalloc(reinterpret_cast<char **>(&c->wfrag[l]), size_t(cnn_packed_bytes(l)))) ||
            (rc = dalloc(&c->bias[l], size_t(cnn_layer_co(l)))))
            return fail(rc);
    // He-normal weights (std sqrt(2 / fan_in)); the output layer is scaled by 0.1 so the
    // initial correction is small; zero biases
    std::vector<float> th(NP, 0.f);
    Rng r{seed};
    for (int l = 0; l < kCnnLayers; ++l) {
        const int ci = cnn_layer_ci(l), co = cnn_layer_co(l);
        const double sd = std::sqrt(2.0 / (9.0 * ci)) * (l == kCnnLayers - 1 ? 0.1 : 1.0);
        float *W = th.data() + cnn_layer_off(l);
        for (int k = 0; k < co * ci * 9; ++k) W[k] = float(sd * r.normal());
    }
    if (hipMemcpy(c->theta, th.data(), NP * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(c->m, 0, NP * sizeof(float)) != hipSuccess || hipMemset(c->v, 0, NP * sizeof(float)) != hipSuccess ||
        hipMemset(c->grad, 0, NP * sizeof(float)) != hipSuccess) {
        set_error("fmgmc_cnn_create: HIP error");
        return fail(FMGMC_EHIP);
    }
    *out = c.release();
    return FMGMC_OK;
}

int fmgmc_cnn_destroy(fmgmc_cnn *c) {
    if (!c) return FMGMC_OK;
    DevGuard g(c->device);
    (void)hipDeviceSynchronize();
    free_train(c);
    dfree(c->theta);
    dfree(c->grad);
    dfree(c->m);
    dfree(c->v);
    for (int l = 0; l < kCnnLayers; ++l) {
        if (c->wfrag[l]) (void)hipFree(c->wfrag[l]);
        dfree(c->bias[l]);
    }
    for (int k = 0; k < 2; ++k)
        if (c->act[k]) (void)hipFree(c->act[k]);
    delete c;
    return FMGMC_OK;
}

int fmgmc_cnn_get_params(const fmgmc_cnn *c, float *theta) {
    if (!c || !theta) {
        set_error("fmgmc_cnn_get_params: bad arguments");
        return FMGMC_EINVAL;
    }
    DevGuard g(c->device);
    FMGMC_HIP(hipMemcpy(theta, c->theta, cnn_nparams() * sizeof(float), hipMemcpyDefault));
    return FMGMC_OK;
}

int fmgmc_cnn_set_params(fmgmc_cnn *c, const float *theta) {
    if (!c || !theta) {
        set_error("fmgmc_cnn_set_params: bad arguments");
        return FMGMC_EINVAL;
    }
    DevGuard g(c->device);
    const size_t bytes = cnn_nparams() * sizeof(float);
    FMGMC_HIP(hipDeviceSynchronize());
    FMGMC_HIP(hipMemcpy(c->theta, theta, bytes, hipMemcpyDefault));
    FMGMC_HIP(hipMemset(c->m, 0, bytes));
    FMGMC_HIP(hipMemset(c->v, 0, bytes));
    c->step = 0;
    c->packed = false;
    return FMGMC_OK;
}

static const char kTag[8] = {'F', 'M', 'G', 'C', 'N', 'N', '0', '1'};

int fmgmc_cnn_save(const fmgmc_cnn *c, const char *path) {
    if (!c || !path) {
        set_error("fmgmc_cnn_save: bad arguments");
        return FMGMC_EINVAL;
    }
    std::vector<float> th(cnn_nparams());
    TRY(fmgmc_cnn_get_params(c, th.data()));
    FILE *f = std::fopen(path, "wb");
    if (!f) {
        set_error(std::string("fmgmc_cnn_save: cannot open ") + path);
        return FMGMC_EINVAL;
    }
    const int32_t hdr[4] = {kCnnIn, kCnnWidth, kCnnRes, 0};
    const bool ok = std::fwrite(kTag, 1, 8, f) == 8 && std::fwrite(hdr, 4, 4, f) == 4 &&
                    std::fwrite(th.data(), 4, th.size(), f) == th.size();
    const bool closed = std::fclose(f) == 0;
    if (!ok || !closed) {
        set_error("fmgmc_cnn_save: write failed");
        return FMGMC_EINVAL;
    }
    return FMGMC_OK;
}

int fmgmc_cnn_load(fmgmc_cnn *c, const char *path) {
    if (!c || !path) {
        set_error("fmgmc_cnn_load: bad arguments");
        return FMGMC_EINVAL;
    }
    FILE *f = std::fopen(path, "rb");
    if (!f) {
        set_error(std::string("fmgmc_cnn_load: cannot open ") + path);
        return FMGMC_EINVAL;
    }
    char tag[8];
    int32_t hdr[4];
    std::vector<float> th(cnn_nparams());
    bool ok = std::fread(tag, 1, 8, f) == 8 && std::memcmp(tag, kTag, 8) == 0 && std::fread(hdr, 4, 4, f) == 4 &&
              hdr[0] == kCnnIn && hdr[1] == kCnnWidth && hdr[2] == kCnnRes &&
              std::fread(th.data(), 4, th.size(), f) == th.size();
    char extra;
    ok = ok && std::fread(&extra, 1, 1, f) == 0;
    std::fclose(f);
    if (!ok) {
        set_error("fmgmc_cnn_load: not a network file of this shape");
        return FMGMC_EINVAL;
    }
    return fmgmc_cnn_set_params(c, th.data());
}

int fmgmc_cnn_forward(fmgmc_cnn *c, int32_t n, int64_t batch, const float *x, float *y, int32_t prec,
                      void *stream) {
    if (!c || !x || !y || (prec != FMGMC_CNN_FP32 && prec != FMGMC_CNN_BF16 && prec != FMGMC_CNN_BF16_FUSED) ||
        (prec == FMGMC_CNN_BF16_FUSED && batch > 65535)) {
        set_error("fmgmc_cnn_forward: bad arguments");
        return FMGMC_EINVAL;
    }
    TRY(check_shape(n, batch));
    DevGuard g(c->device);
    if (!is_dev(x) || !is_dev(y)) {
        set_error("fmgmc_cnn_forward: x and y must be device buffers");
        return FMGMC_EINVAL;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t nn = int64_t(n) * n;
    if (prec == FMGMC_CNN_FP32) {
        TRY(ensure_train(c, batch * nn));
        TRY(forward_f32(c, n, int(batch), x, st));
        FMGMC_HIP(hipMemcpyAsync(y, c->y, batch * nn * sizeof(float), hipMemcpyDeviceToDevice, st));
        return FMGMC_OK;
    }
    TRY(cnn_ensure_packed(c, st));
    if (prec == FMGMC_CNN_BF16_FUSED) {
        InferArgs a{};
        a.n = n;
        a.S = int(batch);
        a.in0 = x;
        a.in1 = x + nn;
        a.in_stride = 2 * nn;
        a.y = y;
        return launch_cnn_fused(a, cnn_packed(c), st);
    }
    const int64_t per = nn * kCnnWidth * 2;  // bytes of one sample's activations
    const int sub = int(std::max<int64_t>(1, std::min<int64_t>(batch, (int64_t(256) << 20) / per)));
    if (c->cap_act < sub * per) {
        FMGMC_HIP(hipStreamSynchronize(st));
        for (int k = 0; k < 2; ++k) {
            if (c->act[k]) (void)hipFree(c->act[k]);
            c->act[k] = nullptr;
        }
        c->cap_act = 0;
        for (int k = 0; k < 2; ++k) TRY(dalloc(reinterpret_cast<char **>(&c->act[k]), size_t(sub * per)));
        c->cap_act = sub * per;
    }
    InferArgs a{};
    a.n = n;
    a.S = int(batch);
    a.in0 = x;
    a.in1 = x + nn;
    a.in_stride = 2 * nn;
    a.log0 = 0;
    a.rr = nullptr;
    a.y = y;
    a.p = nullptr;
    a.active = nullptr;
    return launch_cnn_infer(a, cnn_packed(c), c->act[0], c->act[1], sub, st);
}

int fmgmc_cnn_grad(fmgmc_cnn *c, int32_t n, int64_t batch, const float *x, const float *t, int32_t loss_kind,
                   double *loss, float *grad, void *stream) {
    if (!c || !x || (loss_kind != FMGMC_CNN_LOSS_ERROR && loss_kind != FMGMC_CNN_LOSS_RESIDUAL) ||
        (loss_kind == FMGMC_CNN_LOSS_ERROR && !t)) {
        set_error("fmgmc_cnn_grad: bad arguments");
        return FMGMC_EINVAL;
    }
    TRY(check_shape(n, batch));
    DevGuard g(c->device);
    if (!is_dev(x) || (t && !is_dev(t))) {
        set_error("fmgmc_cnn_grad: x and t must be device buffers");
        return FMGMC_EINVAL;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    double l = 0.0;
    TRY(cnn_grad_impl(c, n, int(batch), x, t, loss_kind, &l, st));
    if (loss) *loss = l;
    if (grad) {
        FMGMC_HIP(hipMemcpyAsync(grad, c->grad, cnn_nparams() * sizeof(float), hipMemcpyDefault, st));
        FMGMC_HIP(hipStreamSynchronize(st));
    }
    return FMGMC_OK;
}

int fmgmc_cnn_adam(fmgmc_cnn *c, double lr, void *stream) {
    if (!c || !(lr >= 0.0)) {
        set_error("fmgmc_cnn_adam: bad arguments");
        return FMGMC_EINVAL;
    }
    DevGuard g(c->device);
    return cnn_adam_impl(c, lr, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
