// Training kernels of the warm-start network, FP32, planar images
// [b][c][y][x]: 3x3 cross-correlation with zero padding (forward, and with
// flipped weights the data gradient), weight gradients as fixed-order
// reductions, the squared-error loss and the Adam update (Kingma and Ba,
// 2015). Also the packing of training pairs from the FMG pass and the
// warm-start judge. Training is off the solve path; these kernels favour
// plain structure (16x16 cell tiles, input channels staged through LDS).
#include <cmath>

#include "cnn.h"

namespace fmgmc {

namespace {

constexpr int TT = 16;  // cells per tile side

template <int CI, int CO, int MODE>
__global__ __launch_bounds__(256) void k_conv_f32(ConvArgs A) {
    constexpr int CB = CI < 8 ? CI : 8;  // input channels per LDS stage
    __shared__ float tile[CB][TT + 2][TT + 3];
    __shared__ float wl[CB][9][CO];
    const int n = A.n, b = blockIdx.z;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int x0 = blockIdx.x * TT, y0 = blockIdx.y * TT;
    const size_t nn = size_t(n) * n;
    const float *in = A.in + size_t(b) * CI * nn;
    float acc[CO];
#pragma unroll
    for (int o = 0; o < CO; ++o) acc[o] = 0.f;
    for (int c0 = 0; c0 < CI; c0 += CB) {
        __syncthreads();
        for (int e = threadIdx.x; e < CB * (TT + 2) * (TT + 2); e += 256) {
            const int c = e / ((TT + 2) * (TT + 2)), r = e % ((TT + 2) * (TT + 2));
            const int yy = r / (TT + 2), xx = r % (TT + 2);
            const int gy = y0 + yy - 1, gx = x0 + xx - 1;
            tile[c][yy][xx] = (gy >= 0 && gy < n && gx >= 0 && gx < n) ? in[(c0 + c) * nn + size_t(gy) * n + gx] : 0.f;
        }
        for (int e = threadIdx.x; e < CB * 9 * CO; e += 256) {
            const int c = e / (9 * CO), t = (e / CO) % 9, o = e % CO;
            wl[c][t][o] = A.W[(o * CI + c0 + c) * 9 + t];
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < CB; ++c)
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const float a = tile[c][ty + t / 3][tx + t % 3];
#pragma unroll
                for (int o = 0; o < CO; ++o) acc[o] += wl[c][t][o] * a;
            }
    }
    const size_t cell = size_t(y0 + ty) * n + x0 + tx;
#pragma unroll
    for (int o = 0; o < CO; ++o) {
        const size_t idx = (size_t(b) * CO + o) * nn + cell;
        if (MODE == CONV_FIRST) {
            const float z = acc[o] + A.bias[o];
            A.out[idx] = z;
            A.out2[idx] = z > 0.f ? z : 0.f;
        } else if (MODE == CONV_RES) {
            const float z = acc[o] + A.bias[o];
            A.out[idx] = z;
            A.out2[idx] = in[o * nn + cell] + (z > 0.f ? z : 0.f);
        } else if (MODE == CONV_OUT) {
            A.out[idx] = acc[o] + A.bias[o];
        } else {
            const float v = acc[o] + (A.addend ? A.addend[idx] : 0.f);
            A.out[idx] = v;
            if (A.out2) A.out2[idx] = A.mask[idx] > 0.f ? v : 0.f;
        }
    }
}

template <int CI, int CO>
__global__ __launch_bounds__(256) void k_wgrad_f32(WgradArgs A) {
    constexpr int COPT = CO >= 8 ? 8 : 1;
    constexpr int NG = CO / COPT;
    constexpr int PAIRS = NG * CI;
    constexpr int SPLIT = 256 / PAIRS;
    static_assert(256 % PAIRS == 0, "thread mapping");
    constexpr int GT = CO * 256;                      // g tile floats
    constexpr int AT = CI * (TT + 2) * (TT + 3);      // a tile floats
    constexpr int SCR = PAIRS * COPT * 10;            // split-reduction scratch
    constexpr int SM = (GT + AT) > SCR ? (GT + AT) : SCR;
    __shared__ float smem[SM];
    float *gt = smem, *at = smem + GT;
    const int t = threadIdx.x, pair = t % PAIRS, split = t / PAIRS;
    const int g = pair % NG, ci = pair / NG;
    const int n = A.n, tpr = n / TT, tiles = A.B * tpr * tpr;
    const size_t nn = size_t(n) * n;
    float acc[COPT][9], bacc[COPT];
#pragma unroll
    for (int o = 0; o < COPT; ++o) {
        bacc[o] = 0.f;
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[o][k] = 0.f;
    }
    for (int tt = blockIdx.x; tt < tiles; tt += gridDim.x) {
        const int b = tt / (tpr * tpr), r = tt % (tpr * tpr);
        const int y0 = (r / tpr) * TT, x0 = (r % tpr) * TT;
        __syncthreads();
        for (int e = t; e < CO * 256; e += 256) {
            const int o = e >> 8, c = e & 255;
            gt[e] = A.g[(size_t(b) * CO + o) * nn + size_t(y0 + (c >> 4)) * n + x0 + (c & 15)];
        }
        for (int e = t; e < CI * (TT + 2) * (TT + 2); e += 256) {
            const int c = e / ((TT + 2) * (TT + 2)), q = e % ((TT + 2) * (TT + 2));
            const int yy = q / (TT + 2), xx = q % (TT + 2), gy = y0 + yy - 1, gx = x0 + xx - 1;
            at[(c * (TT + 2) + yy) * (TT + 3) + xx] =
                (gy >= 0 && gy < n && gx >= 0 && gx < n) ? A.a[(size_t(b) * CI + c) * nn + size_t(gy) * n + gx] : 0.f;
        }
        __syncthreads();
        for (int c = split; c < 256; c += SPLIT) {
            const int cy = c >> 4, cx = c & 15;
            float av[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) av[k] = at[(ci * (TT + 2) + cy + k / 3) * (TT + 3) + cx + k % 3];
#pragma unroll
            for (int o = 0; o < COPT; ++o) {
                const float gv = gt[(g * COPT + o) * 256 + c];
#pragma unroll
                for (int k = 0; k < 9; ++k) acc[o][k] += gv * av[k];
                bacc[o] += gv;
            }
        }
    }
    // fold the SPLIT partial sums of each (co group, ci) pair, in split order
    for (int s = 1; s < SPLIT; ++s) {
        __syncthreads();
        if (split == s) {
#pragma unroll
            for (int o = 0; o < COPT; ++o) {
#pragma unroll
                for (int k = 0; k < 9; ++k) smem[(pair * COPT + o) * 10 + k] = acc[o][k];
                smem[(pair * COPT + o) * 10 + 9] = bacc[o];
            }
        }
        __syncthreads();
        if (split == 0) {
#pragma unroll
            for (int o = 0; o < COPT; ++o) {
#pragma unroll
                for (int k = 0; k < 9; ++k) acc[o][k] += smem[(pair * COPT + o) * 10 + k];
                bacc[o] += smem[(pair * COPT + o) * 10 + 9];
            }
        }
    }
    if (split != 0) return;
    float *out = A.part + size_t(blockIdx.x) * (CO * CI * 9 + CO);
#pragma unroll
    for (int o = 0; o < COPT; ++o) {
        const int co = g * COPT + o;
#pragma unroll
        for (int k = 0; k < 9; ++k) out[(co * CI + ci) * 9 + k] = acc[o][k];
        if (ci == 0) out[CO * CI * 9 + co] = bacc[o];
    }
}

__global__ void k_sum_parts(const float *part, int P, int64_t np, float *out) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= np) return;
    double s = 0.0;
    for (int p = 0; p < P; ++p) s += double(part[size_t(p) * np + k]);
    out[k] = float(s);
}

__global__ void k_flip(const float *W, int ci, int co, float *Wt) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ci * co * 9) return;
    const int o = e / (ci * 9), c = (e / 9) % ci, t = e % 9;
    Wt[(c * co + o) * 9 + (8 - t)] = W[e];
}

constexpr int kMseBlocks = 256;

__global__ __launch_bounds__(256) void k_mse(const float *y, const float *t, int64_t N, float *dy, double *part) {
    __shared__ double red[4];
    double s = 0.0;
    const double inv = 1.0 / double(N);
    for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < N; k += int64_t(gridDim.x) * 256) {
        const double d = double(y[k]) - double(t[k]);
        s += d * d;
        dy[k] = float(2.0 * d * inv);
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ void k_mse_final(const double *part, int P, int64_t N, double *loss) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int p = 0; p < P; ++p) s += part[p];
    loss[0] = s / double(N);
}

// (A v) at cell (i, j) of sample image v, A the stage operator from K = exp(x0):
// harmonic interior faces, 2K on the west/east Dirichlet faces, no flow north/south
__device__ __forceinline__ float apply_at(int n, const float *x0, const float *v, int i, int j) {
    const int P = j * n + i;
    const float kp = __expf(x0[P]), vp = v[P];
    float acc = 0.f;
    auto face = [&](int Q) {
        const float kq = __expf(x0[Q]);
        acc += (2.f * kp * kq / (kp + kq)) * (vp - v[Q]);
    };
    if (i > 0) face(P - 1);
    else acc += 2.f * kp * vp;
    if (i < n - 1) face(P + 1);
    else acc += 2.f * kp * vp;
    if (j > 0) face(P - n);
    if (j < n - 1) face(P + n);
    return acc;
}

// residual loss, first pass: u = x1 - A y; block partial sums of u^2
__global__ __launch_bounds__(256) void k_resid_u(int n, int64_t total, const float *x, const float *y, float *u,
                                                 double *part) {
    __shared__ double red[4];
    const int64_t nn = int64_t(n) * n;
    double s = 0.0;
    for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < total; k += int64_t(gridDim.x) * 256) {
        const int64_t b = k / nn;
        const int c = int(k % nn);
        const float *x0 = x + 2 * b * nn;
        const float v = x0[nn + c] - apply_at(n, x0, y + b * nn, c % n, c / n);
        u[k] = v;
        s += double(v) * v;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// second pass: dL/dy = -2 A u / N (A is symmetric)
__global__ void k_resid_dy(int n, int64_t total, const float *x, const float *u, float *dy, float scale) {
    const int64_t nn = int64_t(n) * n;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= total) return;
    const int64_t b = k / nn;
    const int c = int(k % nn);
    dy[k] = scale * apply_at(n, x + 2 * b * nn, u + b * nn, c % n, c / n);
}

__global__ void k_adam(float *theta, const float *g, float *m, float *v, int64_t np, double lr, double b1,
                       double b2, double eps, double c1, double c2) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= np) return;
    const double gk = g[k];
    const double mk = b1 * double(m[k]) + (1.0 - b1) * gk;
    const double vk = b2 * double(v[k]) + (1.0 - b2) * gk * gk;
    m[k] = float(mk);
    v[k] = float(vk);
    theta[k] = float(double(theta[k]) - lr * (mk / c1) / (sqrt(vk / c2) + eps));
}

__device__ __forceinline__ double inv_rms(const double *rr, int s, int n) {
    const double r = rr[s];
    return r > 0.0 ? 1.0 / sqrt(r / (double(n) * n)) : 0.0;
}

__global__ void k_pack_x(int n, const float *K, const float *r, const double *rr, float *x) {
    const int s = blockIdx.y;
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x, nn = int64_t(n) * n;
    if (c >= nn) return;
    const double ir = inv_rms(rr, s, n);
    x[(2 * s) * nn + c] = logf(K[s * nn + c]);
    x[(2 * s + 1) * nn + c] = float(double(r[s * nn + c]) * ir);
}

__global__ void k_pack_t(int n, const double *p, const double *p0, const double *rr, float *t) {
    const int s = blockIdx.y;
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x, nn = int64_t(n) * n;
    if (c >= nn) return;
    t[s * nn + c] = float((p[s * nn + c] - p0[s * nn + c]) * inv_rms(rr, s, n));
}

__global__ void k_judge(int S, const double *rr_new, const double *rr_old, int32_t *restore, uint8_t *flags) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const bool keep = rr_new[s] < rr_old[s];  // false for NaN too
    restore[s] = keep ? 0 : 1;
    if (!keep) flags[s] |= FMGMC_FLAG_WARM_REJECTED;
}

__global__ void k_copy_f64(const double *src, double *dst, int64_t n) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = src[k];
}

int last_error() { return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP; }

template <int CI, int CO, int MODE>
int conv_launch(const ConvArgs &a, dim3 g, hipStream_t st) {
    hipLaunchKernelGGL((k_conv_f32<CI, CO, MODE>), g, dim3(256), 0, st, a);
    return last_error();
}

}  // namespace

int launch_conv_f32(int ci, int co, int mode, const ConvArgs &a, hipStream_t st) {
    if (a.n < TT || a.n % TT || a.B < 1) {
        set_error("launch_conv_f32: n must be a multiple of 16");
        return FMGMC_EINVAL;
    }
    const dim3 g(a.n / TT, a.n / TT, a.B);
    if (ci == kCnnIn && co == kCnnWidth && mode == CONV_FIRST) return conv_launch<kCnnIn, kCnnWidth, CONV_FIRST>(a, g, st);
    if (ci == kCnnWidth && co == kCnnWidth && mode == CONV_RES)
        return conv_launch<kCnnWidth, kCnnWidth, CONV_RES>(a, g, st);
    if (ci == kCnnWidth && co == kCnnWidth && mode == CONV_BWD)
        return conv_launch<kCnnWidth, kCnnWidth, CONV_BWD>(a, g, st);
    if (ci == kCnnWidth && co == 1 && mode == CONV_OUT) return conv_launch<kCnnWidth, 1, CONV_OUT>(a, g, st);
    if (ci == 1 && co == kCnnWidth && mode == CONV_BWD) return conv_launch<1, kCnnWidth, CONV_BWD>(a, g, st);
    set_error("launch_conv_f32: unsupported layer shape");
    return FMGMC_EINVAL;
}

int launch_wgrad_f32(int ci, int co, const WgradArgs &a, hipStream_t st) {
    if (a.n < TT || a.n % TT || a.P < 1) {
        set_error("launch_wgrad_f32: bad shape");
        return FMGMC_EINVAL;
    }
    if (ci == kCnnWidth && co == kCnnWidth)
        hipLaunchKernelGGL((k_wgrad_f32<kCnnWidth, kCnnWidth>), dim3(a.P), dim3(256), 0, st, a);
    else if (ci == kCnnIn && co == kCnnWidth)
        hipLaunchKernelGGL((k_wgrad_f32<kCnnIn, kCnnWidth>), dim3(a.P), dim3(256), 0, st, a);
    else if (ci == kCnnWidth && co == 1)
        hipLaunchKernelGGL((k_wgrad_f32<kCnnWidth, 1>), dim3(a.P), dim3(256), 0, st, a);
    else {
        set_error("launch_wgrad_f32: unsupported layer shape");
        return FMGMC_EINVAL;
    }
    return last_error();
}

int launch_sum_parts(const float *part, int P, int64_t np, float *out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_parts, dim3((np + 255) / 256), dim3(256), 0, st, part, P, np, out);
    return last_error();
}

int launch_flip_weights(const float *W, int ci, int co, float *Wt, hipStream_t st) {
    hipLaunchKernelGGL(k_flip, dim3((ci * co * 9 + 255) / 256), dim3(256), 0, st, W, ci, co, Wt);
    return last_error();
}

int launch_mse(const float *y, const float *t, int64_t N, float *dy, double *part, double *loss, hipStream_t st) {
    hipLaunchKernelGGL(k_mse, dim3(kMseBlocks), dim3(256), 0, st, y, t, N, dy, part);
    hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(64), 0, st, part, kMseBlocks, N, loss);
    return last_error();
}

int launch_resid_loss(int n, int B, const float *x, const float *y, float *u, float *dy, double *part,
                      double *loss, hipStream_t st) {
    const int64_t total = int64_t(B) * n * n;
    hipLaunchKernelGGL(k_resid_u, dim3(kMseBlocks), dim3(256), 0, st, n, total, x, y, u, part);
    hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(64), 0, st, part, kMseBlocks, total, loss);
    hipLaunchKernelGGL(k_resid_dy, dim3((total + 255) / 256), dim3(256), 0, st, n, total, x, u, dy,
                       float(-2.0 / double(total)));
    return last_error();
}

int launch_adam(float *theta, const float *g, float *m, float *v, int64_t np, double lr, double b1, double b2,
                double eps, int step, hipStream_t st) {
    const double c1 = 1.0 - std::pow(b1, step), c2 = 1.0 - std::pow(b2, step);
    hipLaunchKernelGGL(k_adam, dim3((np + 255) / 256), dim3(256), 0, st, theta, g, m, v, np, lr, b1, b2, eps, c1, c2);
    return last_error();
}

int launch_pack_x(int n, int S, const float *K, const float *r, const double *rr, float *x, hipStream_t st) {
    if (S <= 0) return FMGMC_OK;
    hipLaunchKernelGGL(k_pack_x, dim3((n * n + 255) / 256, S), dim3(256), 0, st, n, K, r, rr, x);
    return last_error();
}

int launch_pack_t(int n, int S, const double *p, const double *p0, const double *rr, float *t, hipStream_t st) {
    if (S <= 0) return FMGMC_OK;
    hipLaunchKernelGGL(k_pack_t, dim3((n * n + 255) / 256, S), dim3(256), 0, st, n, p, p0, rr, t);
    return last_error();
}

int launch_judge(int S, const double *rr_new, const double *rr_old, int32_t *restore, uint8_t *flags,
                 hipStream_t st) {
    if (S <= 0) return FMGMC_OK;
    hipLaunchKernelGGL(k_judge, dim3((S + 255) / 256), dim3(256), 0, st, S, rr_new, rr_old, restore, flags);
    return last_error();
}

int launch_copy_f64(const double *src, double *dst, int64_t n, hipStream_t st) {
    if (n <= 0) return FMGMC_OK;
    hipLaunchKernelGGL(k_copy_f64, dim3((n + 255) / 256), dim3(256), 0, st, src, dst, n);
    return last_error();
}

}  // namespace fmgmc
