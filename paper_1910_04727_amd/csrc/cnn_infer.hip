// BF16 inference of the warm-start network on the matrix cores of gfx950
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation). One launch per layer;
// activations are channel-last bf16 [s][y][x][32] (64 B per cell), so an MFMA
// A fragment (16 cells x 8 channels per 16-lane group) is one 16-byte LDS read.
//
// Workgroup: 4 waves, an output tile of 4 rows x TW cells (TW = min(64, n));
// wave w owns row w, i.e. TW/16 M-tiles of 16 cells, and both 16-channel
// N-tiles. The input rows y0-1 .. y0+4 (plus one halo cell each side) are
// staged in LDS with an 80-byte cell stride (spreads the 16-byte reads of a
// 16-lane group over distinct banks). The 3x3 convolution is 9 taps x K = 32
// input channels: per tap one B fragment per N-tile (pre-packed weights,
// 16 bytes per lane from L2) and one MFMA per (M-tile, N-tile).
//
// First layer (2 -> 32): the 2 channels x 9 taps = 18 products fit one K = 32
// MFMA (k = 2 tap + channel, k >= 18 zero); its inputs are FP32 planes (log K
// and the residual scaled by 1 / rms(r)), converted to bf16 in the A fragment.
// Last layer (32 -> 1): one N-tile whose column 0 holds the output; the
// epilogue writes y or applies the correction p += rms(r) * y in FP64.
#include <cmath>

#include "cnn.h"

namespace fmgmc {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int CH = kCnnWidth;   // 32 channels
constexpr int CS = 40;          // LDS cell stride in bf16 (80 bytes)
constexpr int ROWS = 4;         // output rows per workgroup (one per wave)
constexpr int IR = ROWS + 2;    // staged input rows

enum { L_FIRST = 0, L_MID = 1, L_LAST = 2 };

struct LayerArgs {
    int n, s0;
    const __bf16 *in;      // [sub][n][n][32] (MID, LAST)
    __bf16 *out;           // [sub][n][n][32] (FIRST, MID)
    const bf8 *w;          // fragments: FIRST [2][64], MID [9][2][64], LAST [9][64]
    const float *bias;     // [32] or [1]
    // FIRST inputs (sample s = s0 + blockIdx.z)
    const float *in0, *in1;
    int64_t in_stride;
    int log0;
    const double *rr;      // nullable
    // LAST outputs
    float *y;
    double *p;
    const int32_t *active;
};

__device__ __forceinline__ double scale_of(const double *rr, int s, int n) {
    if (!rr) return 1.0;
    const double r = rr[s];
    return r > 0.0 ? sqrt(r / (double(n) * n)) : 0.0;
}

template <int TW, int KIND>
__global__ __launch_bounds__(256) void k_cnn_layer(LayerArgs A) {
    constexpr int MT = TW / 16;                    // M-tiles per wave
    constexpr int NT = (KIND == L_LAST) ? 1 : 2;   // N-tiles
    constexpr int TILE = IR * (TW + 2) * CS;       // bf16 elements
    __shared__ __attribute__((aligned(16))) __bf16 tile[TILE];
    __shared__ float xin[IR * (TW + 2) * 2];       // FIRST: FP32 input planes
    const int n = A.n, sl = blockIdx.z, s = A.s0 + sl;
    if (A.active && A.active[s] == 0) return;
    const int x0 = blockIdx.x * TW, y0 = blockIdx.y * ROWS;
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const size_t nn = size_t(n) * n;

    // ---- stage inputs
    if (KIND == L_FIRST) {
        const double sc = scale_of(A.rr, s, n);
        const float inv = sc > 0.0 ? float(1.0 / sc) : 0.f;
        const float *p0 = A.in0 + size_t(s) * A.in_stride, *p1 = A.in1 + size_t(s) * A.in_stride;
        for (int e = t; e < IR * (TW + 2); e += 256) {
            const int r = e / (TW + 2), c = e % (TW + 2), gy = y0 - 1 + r, gx = x0 - 1 + c;
            float a = 0.f, b = 0.f;
            if (gy >= 0 && gy < n && gx >= 0 && gx < n) {
                const size_t o = size_t(gy) * n + gx;
                a = A.log0 ? __logf(p0[o]) : p0[o];
                b = A.rr ? p1[o] * inv : p1[o];
            }
            xin[2 * e] = a;
            xin[2 * e + 1] = b;
        }
    } else {
        const __bf16 *src = A.in + size_t(sl) * nn * CH;
        for (int e = t; e < IR * (TW + 2) * 4; e += 256) {
            const int part = e & 3, c = (e >> 2) % (TW + 2), r = (e >> 2) / (TW + 2);
            const int gy = y0 - 1 + r, gx = x0 - 1 + c;
            uint4 v = {0u, 0u, 0u, 0u};
            if (gy >= 0 && gy < n && gx >= 0 && gx < n)
                v = *reinterpret_cast<const uint4 *>(src + (size_t(gy) * n + gx) * CH + 8 * part);
            *reinterpret_cast<uint4 *>(tile + (r * (TW + 2) + c) * CS + 8 * part) = v;
        }
    }
    __syncthreads();

    // ---- contraction
    f4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int q = 0; q < NT; ++q) acc[m][q] = f4{0.f, 0.f, 0.f, 0.f};
    if (KIND == L_FIRST) {
        const bf8 b0 = A.w[l], b1 = A.w[64 + l];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            bf8 a;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 8 * (l >> 4) + e;
                float v = 0.f;
                if (k < 18) {
                    const int tap = k >> 1;
                    v = xin[2 * ((w + tap / 3) * (TW + 2) + 16 * m + (l & 15) + tap % 3) + (k & 1)];
                }
                a[e] = __bf16(v);
            }
            acc[m][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0, acc[m][0], 0, 0, 0);
            acc[m][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, acc[m][1], 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            bf8 b[NT];
#pragma unroll
            for (int q = 0; q < NT; ++q) b[q] = A.w[(tap * NT + q) * 64 + l];
            const int dy = tap / 3, dx = tap % 3;
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                const bf8 a = *reinterpret_cast<const bf8 *>(tile + ((w + dy) * (TW + 2) + 16 * m + (l & 15) + dx) * CS +
                                                            8 * (l >> 4));
#pragma unroll
                for (int q = 0; q < NT; ++q)
                    acc[m][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[q], acc[m][q], 0, 0, 0);
            }
        }
    }

    // ---- epilogue. D layout: lane l, register v -> cell 16 m + 4 (l / 16) + v, channel 16 q + l % 16
    if (KIND == L_LAST) {
        if ((l & 15) != 0) return;
        const float b0 = A.bias[0];
        const double sc = scale_of(A.rr, s, n);
        const int gy = y0 + w;
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gx = x0 + 16 * m + 4 * (l >> 4) + v;
                const size_t o = size_t(s) * nn + size_t(gy) * n + gx;
                const float yv = acc[m][0][v] + b0;
                if (A.y) A.y[o] = yv;
                if (A.p) A.p[o] += sc * double(yv);
            }
        return;
    }
    float res[MT][NT][4];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const int co = 16 * q + (l & 15);
            const float bq = A.bias[co];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float z = acc[m][q][v] + bq;
                z = z > 0.f ? z : 0.f;
                if (KIND == L_MID) {
                    const int c = 16 * m + 4 * (l >> 4) + v;
                    z += float(tile[((w + 1) * (TW + 2) + c + 1) * CS + co]);
                }
                res[m][q][v] = z;
            }
        }
    __syncthreads();  // the input tile is reused as the output tile [ROWS][TW][32]
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int q = 0; q < NT; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                tile[(w * TW + 16 * m + 4 * (l >> 4) + v) * CH + 16 * q + (l & 15)] = __bf16(res[m][q][v]);
    __syncthreads();
    __bf16 *dst = A.out + size_t(sl) * nn * CH;
    for (int e = t; e < ROWS * TW * 4; e += 256) {
        const int part = e & 3, c = (e >> 2) % TW, r = (e >> 2) / TW;
        *reinterpret_cast<uint4 *>(dst + (size_t(y0 + r) * n + x0 + c) * CH + 8 * part) =
            *reinterpret_cast<const uint4 *>(tile + (r * TW + c) * CH + 8 * part);
    }
}

// Fragment packing from the FP32 parameter vector (layout of cnn.h).
__global__ void k_pack_first(const float *W, bf8 *frag) {
    const int l = threadIdx.x & 63, q = threadIdx.x >> 6;  // 128 threads
    bf8 v;
    for (int e = 0; e < 8; ++e) {
        const int k = 8 * (l >> 4) + e, co = 16 * q + (l & 15);
        float x = 0.f;
        if (k < 18) x = W[(co * kCnnIn + (k & 1)) * 9 + (k >> 1)];
        v[e] = __bf16(x);
    }
    frag[q * 64 + l] = v;
}

__global__ void k_pack_mid(const float *W, bf8 *frag, int nt) {
    const int l = threadIdx.x & 63, f = blockIdx.x;  // f = tap * nt + q
    const int tap = f / nt, q = f % nt, co = 16 * q + (l & 15);
    bf8 v;
    for (int e = 0; e < 8; ++e) {
        const int ci = 8 * (l >> 4) + e;
        float x = 0.f;
        if (nt == 2 || co == 0) x = W[(co * CH + ci) * 9 + tap];
        v[e] = __bf16(x);
    }
    frag[f * 64 + l] = v;
}

__global__ void k_copy_f32(const float *src, float *dst, int n) {
    const int k = threadIdx.x;
    if (k < n) dst[k] = src[k];
}

template <int TW>
int run_layers(const InferArgs &a, const CnnPacked &w, void *act0, void *act1, int sub, hipStream_t st) {
    const int n = a.n;
    __bf16 *b0 = static_cast<__bf16 *>(act0), *b1 = static_cast<__bf16 *>(act1);
    for (int s0 = 0; s0 < a.S; s0 += sub) {
        const int cnt = std::min(sub, a.S - s0);
        const dim3 grid(n / TW, n / ROWS, cnt);
        LayerArgs L{};
        L.n = n;
        L.s0 = s0;
        L.active = a.active;
        L.rr = a.rr;
        L.in0 = a.in0;
        L.in1 = a.in1;
        L.in_stride = a.in_stride;
        L.log0 = a.log0;
        L.out = b0;
        L.w = static_cast<const bf8 *>(w.w[0]);
        L.bias = w.b[0];
        hipLaunchKernelGGL((k_cnn_layer<TW, L_FIRST>), grid, dim3(256), 0, st, L);
        __bf16 *cur = b0, *nxt = b1;
        for (int k = 1; k <= kCnnRes; ++k) {
            L.in = cur;
            L.out = nxt;
            L.w = static_cast<const bf8 *>(w.w[k]);
            L.bias = w.b[k];
            hipLaunchKernelGGL((k_cnn_layer<TW, L_MID>), grid, dim3(256), 0, st, L);
            std::swap(cur, nxt);
        }
        L.in = cur;
        L.out = nullptr;
        L.w = static_cast<const bf8 *>(w.w[kCnnLayers - 1]);
        L.bias = w.b[kCnnLayers - 1];
        L.y = a.y;
        L.p = a.p;
        hipLaunchKernelGGL((k_cnn_layer<TW, L_LAST>), grid, dim3(256), 0, st, L);
    }
    return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP;
}

}  // namespace

int cnn_packed_bytes(int layer) {
    if (layer == 0) return 2 * 64 * 16;
    if (layer == kCnnLayers - 1) return 9 * 64 * 16;
    return 9 * 2 * 64 * 16;
}

int launch_pack_weights(const float *theta, void *const *wfrag, float *const *bias, hipStream_t st) {
    for (int l = 0; l < kCnnLayers; ++l) {
        const float *W = theta + cnn_layer_off(l);
        const int co = cnn_layer_co(l), ci = cnn_layer_ci(l);
        if (l == 0)
            hipLaunchKernelGGL(k_pack_first, dim3(1), dim3(128), 0, st, W, static_cast<bf8 *>(wfrag[l]));
        else
            hipLaunchKernelGGL(k_pack_mid, dim3(9 * (co == 1 ? 1 : 2)), dim3(64), 0, st, W,
                               static_cast<bf8 *>(wfrag[l]), co == 1 ? 1 : 2);
        hipLaunchKernelGGL(k_copy_f32, dim3(1), dim3(64), 0, st, W + size_t(co) * ci * 9, bias[l], co);
    }
    return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP;
}

int launch_cnn_infer(const InferArgs &a, const CnnPacked &w, void *act0, void *act1, int sub_batch,
                     hipStream_t st) {
    const int n = a.n;
    if (n < 16 || (n & (n - 1)) || n > 1024 || sub_batch < 1) {
        set_error("launch_cnn_infer: n must be a power of two in [16, 1024]");
        return FMGMC_EINVAL;
    }
    if (a.S <= 0) return FMGMC_OK;
    if (n == 16) return run_layers<16>(a, w, act0, act1, sub_batch, st);
    if (n == 32) return run_layers<32>(a, w, act0, act1, sub_batch, st);
    return run_layers<64>(a, w, act0, act1, sub_batch, st);
}

}  // namespace fmgmc
