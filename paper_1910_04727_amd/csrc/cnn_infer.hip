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
// Storage order of a cell's 32 channels (in HBM and in LDS): position
// 8 g + 4 q + v holds channel 16 q + 4 g + v (g < 4, q < 2, v < 4). In the
// fused kernel's D layout lane l holds channels 16 q + 4 (l / 16) + v of a
// cell, so its eight values are one 16-byte word and its epilogue stores and
// residual reads are single 16-byte accesses (conflict-free at the 80-byte
// cell stride; 8-byte ones two-way conflicted). The input-channel order of
// the packed weights follows, so every contraction runs over the positions.
__host__ __device__ constexpr int cnn_pos(int c) { return 8 * ((c >> 2) & 3) + 4 * (c >> 4) + (c & 3); }
__host__ __device__ constexpr int cnn_chan(int p) { return 16 * ((p >> 2) & 1) + 4 * (p >> 3) + (p & 3); }
static_assert(cnn_chan(cnn_pos(21)) == 21 && cnn_pos(cnn_chan(13)) == 13, "channel order");
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
                    z += float(tile[((w + 1) * (TW + 2) + c + 1) * CS + cnn_pos(co)]);
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
                tile[(w * TW + 16 * m + 4 * (l >> 4) + v) * CH + cnn_pos(16 * q + (l & 15))] = __bf16(res[m][q][v]);
    __syncthreads();
    __bf16 *dst = A.out + size_t(sl) * nn * CH;
    for (int e = t; e < ROWS * TW * 4; e += 256) {
        const int part = e & 3, c = (e >> 2) % TW, r = (e >> 2) / TW;
        *reinterpret_cast<uint4 *>(dst + (size_t(y0 + r) * n + x0 + c) * CH + 8 * part) =
            *reinterpret_cast<const uint4 *>(tile + (r * TW + c) * CH + 8 * part);
    }
}

// ---------------------------------------------------------------------------
// All six layers in one pass. A workgroup marches up a strip of FW = 64
// computed columns of one sample (FV = 52 valid output columns: each layer
// narrows the valid region by one cell per side), with every layer's
// activations for the rows in flight in LDS: a 4-row ring per hidden layer
// ([row][1 + 64 + 1 cells][32 channels] bf16, an 80-byte cell stride as in
// k_cnn_layer) and a 4-row ring of the two FP32 input planes. Layer k works on
// row F - 2k at step F, two rows behind layer k - 1, so every row it reads was
// written in an earlier step and one barrier per step orders the whole
// pipeline. Eight waves: a pair per layer group, each wave of a pair taking
// two of the four M-tiles, with the group's B fragments in registers for the
// whole strip (pair 0: layers 0 and 1; pair 1: layer 2; pair 2: layer 3;
// pair 3: layer 4; pairs 1 and 2 also take one M-tile each of the output
// layer). Cells outside the domain are stored as zeros (the zero padding of
// every convolution), so activations never leave the chip. The input planes
// are loaded four rows ahead; the output is stored, never read back. The
// fragments, the tap order and the bf16 rounding points are those of
// k_cnn_layer, so the network output y is the same bits.
constexpr int FW = 64;                 // computed cells per strip row
constexpr int FV = FW - 12;            // valid output cells per strip
constexpr int FROW = (FW + 2) * CS;    // bf16 elements of one ring row (pad cell each side)
constexpr int FRING = 4 * FROW;        // one layer's ring
constexpr int FPRE = 2;                // input rows in flight
constexpr size_t fused_lds_bytes() {
    return size_t(kCnnRes + 1) * FRING * sizeof(__bf16) + size_t(4) * (FW + 2) * 2 * sizeof(float);
}

struct FusedArgs {
    int n;
    const float *in0, *in1;
    int64_t in_stride;
    int log0;
    const double *rr;
    float *y;   // network output (nullable)
    float *e;   // rms(r) * output in FP32 (nullable): the correction of the start
    const int32_t *active;
    const bf8 *w[kCnnLayers];
    const float *bias[kCnnLayers];
};

__global__ __launch_bounds__(512) void k_cnn_fused(FusedArgs A) {
    const int n = A.n, s = blockIdx.y;
    if (A.active && A.active[s] == 0) return;
    extern __shared__ __attribute__((aligned(16))) unsigned char fsm[];
    __bf16 *ring = reinterpret_cast<__bf16 *>(fsm);                                    // [5][4][66][CS]
    float *xin = reinterpret_cast<float *>(fsm + size_t(kCnnRes + 1) * FRING * sizeof(__bf16));  // [4][66][2]
    const int t = threadIdx.x, wv = t >> 6, role = wv >> 1, half = wv & 1, l = t & 63;
    const int gx0 = int(blockIdx.x) * FV - 6;  // global column of computed cell 0
    const size_t nn = size_t(n) * n;
    for (size_t e = t; e < fused_lds_bytes() / 16; e += 512) reinterpret_cast<uint4 *>(fsm)[e] = uint4{0u, 0u, 0u, 0u};
    // this wave's weights: wa the hidden layer role + 1; wb layer 0 (role 0, entries 0 and 1)
    // or the output layer (roles 1, 2)
    bf8 wa[18], wb[9];
    const int la = role + 1;
#pragma unroll
    for (int f = 0; f < 18; ++f) wa[f] = A.w[la][f * 64 + l];
#pragma unroll
    for (int f = 0; f < 9; ++f)
        wb[f] = role == 0 ? (f < 2 ? A.w[0][f * 64 + l] : bf8{})
                          : ((role == 1 || role == 2) ? A.w[kCnnLayers - 1][f * 64 + l] : bf8{});
    const float bo = A.bias[kCnnLayers - 1][0];
    const double sc = scale_of(A.rr, s, n);
    const float inv = sc > 0.0 ? float(1.0 / sc) : 0.f;
    // input planes: thread t < 128 owns channel t / 64 of computed cell t % 64
    const int ich = t >> 6, ic = t & 63, igc = gx0 + ic;
    const bool icol = t < 128 && igc >= 0 && igc < n;
    const float *ip = (ich == 0 ? A.in0 : A.in1) + size_t(s) * A.in_stride;
    auto load_raw = [&](int row) -> float { return (icol && row >= 0 && row < n) ? ip[size_t(row) * n + igc] : 0.f; };
    // the network input of a loaded value (0 outside the domain: zero padding)
    auto input = [&](float v, int row) -> float {
        if (!icol || row < 0 || row >= n) return 0.f;
        return ich == 0 ? (A.log0 ? __logf(v) : v) : (A.rr ? v * inv : v);
    };
    __syncthreads();
    if (t < 128) xin[(ic + 1) * 2 + ich] = input(load_raw(0), 0);  // row 0 in slot 0
    // queue of raw input rows in flight: qu holds row F + u + 1 at step F + u (F a multiple of FPRE)
    float q0 = load_raw(1), q1 = load_raw(2);
    __syncthreads();

    // Products with the weights as the A operand (rows = output channels) and the
    // activations as B (columns = cells): the packed fragments serve either
    // operand, and D then gives each lane four consecutive channels of one cell
    // (lane l, register v -> channel 16 q + 4 (l / 16) + v, cell 16 m + l % 16),
    // so the epilogue reads the residual and writes the result 8 bytes at a time.
    // Biases of this lane's channels: 16 q + 4 (l / 16) + v.
    float bz[2][4], ba[2][4];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            bz[q][v] = A.bias[0][16 * q + 4 * (l >> 4) + v];
            ba[q][v] = A.bias[la][16 * q + 4 * (l >> 4) + v];
        }
    // hidden layer k on row r (cell tiles 2 half, 2 half + 1) from ring k - 1 into
    // ring k (k >= 1), or layer 0 from the input planes
    auto hidden = [&](int k, int r, const bf8 *wk, const float (*bk)[4]) {
        __bf16 *dst = ring + k * FRING + (r & 3) * FROW;
        if (r < 0 || r >= n) {  // zero padding of the next layer's input (each wave its half of the row)
            for (int e = l + 64 * half; e < FROW / 8; e += 128) reinterpret_cast<uint4 *>(dst)[e] = uint4{0u, 0u, 0u, 0u};
            return;
        }
        f4 acc[2][2];  // [channel tile q][cell tile m]
#pragma unroll
        for (int m = 0; m < 2; ++m) acc[0][m] = acc[1][m] = f4{0.f, 0.f, 0.f, 0.f};
        if (k == 0) {
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                bf8 a;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int kk = 8 * (l >> 4) + e;
                    float v = 0.f;
                    if (kk < 18) {
                        const int tap = kk >> 1;
                        v = xin[(((r + tap / 3 - 1) & 3) * (FW + 2) + 16 * (2 * half + m) + (l & 15) + tap % 3) * 2 + (kk & 1)];
                    }
                    a[e] = __bf16(v);
                }
                acc[0][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wk[0], a, acc[0][m], 0, 0, 0);
                acc[1][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wk[1], a, acc[1][m], 0, 0, 0);
            }
        } else {
            const __bf16 *src = ring + (k - 1) * FRING;
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const __bf16 *srow = src + ((r + tap / 3 - 1) & 3) * FROW;
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    const bf8 a = *reinterpret_cast<const bf8 *>(srow + (16 * (2 * half + m) + (l & 15) + tap % 3) * CS +
                                                                8 * (l >> 4));
                    acc[0][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wk[2 * tap], a, acc[0][m], 0, 0, 0);
                    acc[1][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wk[2 * tap + 1], a, acc[1][m], 0, 0, 0);
                }
            }
        }
        // epilogue: bias, ReLU, the residual (k >= 1), zeros outside the domain; the
        // lane's channels 16 q + 4 (l / 16) + v sit at positions 8 (l / 16) + 4 q + v
        const __bf16 *res = ring + (k > 0 ? k - 1 : 0) * FRING + (r & 3) * FROW;
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const int c = 16 * (2 * half + m) + (l & 15), gc = gx0 + c;
            const bool in = gc >= 0 && gc < n;
            const int pos = (c + 1) * CS + 8 * (l >> 4);
            bf8 rv = bf8{};
            if (k > 0) rv = *reinterpret_cast<const bf8 *>(res + pos);
            bf8 out;
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    float z = acc[q][m][v] + bk[q][v];
                    z = z > 0.f ? z : 0.f;
                    if (k > 0) z += float(rv[4 * q + v]);
                    out[4 * q + v] = __bf16(in ? z : 0.f);
                }
            *reinterpret_cast<bf8 *>(dst + pos) = out;
        }
    };
    // output layer on row r for cell tile m (one channel tile; channel 0 is the output,
    // held by lanes 0..15 in register 0)
    auto output = [&](int r, int m) {
        if (r < 0 || r >= n) return;
        const __bf16 *src = ring + kCnnRes * FRING;
        f4 acc = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const __bf16 *srow = src + ((r + tap / 3 - 1) & 3) * FROW;
            const bf8 a = *reinterpret_cast<const bf8 *>(srow + (16 * m + (l & 15) + tap % 3) * CS + 8 * (l >> 4));
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb[tap], a, acc, 0, 0, 0);
        }
        if (l >= 16) return;
        const int c = 16 * m + l, gc = gx0 + c;
        if (c < 6 || c >= 6 + FV || gc >= n) return;
        const size_t o = size_t(s) * nn + size_t(r) * n + gc;
        const float yv = acc[0] + bo;
        if (A.y) A.y[o] = yv;
        if (A.e) A.e[o] = float(sc * double(yv));
    };
    const int last = n - 1 + 2 * (kCnnLayers - 1);
    for (int F = 0; F <= last; F += FPRE) {
        // FPRE steps per iteration so that the input queue slots are constants:
        // at step F + u the queue slot q_u holds row F + u + 1 and takes row F + u + 1 + FPRE
#define FMGMC_FUSED_STEP(u, qv)                                                                     \
        if (F + u <= last) {                                                                         \
            const int Fs = F + u;                                                                    \
            if (t < 128) xin[((((Fs + 1) & 3) * (FW + 2)) + ic + 1) * 2 + ich] = input(qv, Fs + 1); \
            qv = load_raw(Fs + 1 + FPRE);                                                            \
            __syncthreads();                                                                         \
            if (role == 0) {                                                                         \
                hidden(0, Fs, wb, bz);                                                               \
                hidden(1, Fs - 2, wa, ba);                                                           \
            } else {                                                                                 \
                hidden(la, Fs - 2 * la, wa, ba);                                                     \
                if (role == 1) output(Fs - 2 * (kCnnLayers - 1), half);                              \
                if (role == 2) output(Fs - 2 * (kCnnLayers - 1), 2 + half);                          \
            }                                                                                        \
        }
        FMGMC_FUSED_STEP(0, q0)
        FMGMC_FUSED_STEP(1, q1)
#undef FMGMC_FUSED_STEP
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
        const int ci = cnn_chan(8 * (l >> 4) + e);  // the input channel at that storage position
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

int launch_cnn_fused(const InferArgs &a, const CnnPacked &w, hipStream_t st) {
    const int n = a.n;
    if (n < 16 || (n & (n - 1)) || n > 1024 || a.S > 65535) {
        set_error("launch_cnn_fused: n must be a power of two in [16, 1024], at most 65535 samples");
        return FMGMC_EINVAL;
    }
    if (a.S <= 0) return FMGMC_OK;
    static bool attr_set = false;  // the kernel's LDS exceeds the default dynamic limit
    if (!attr_set) {
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_cnn_fused),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(fused_lds_bytes())) != hipSuccess) {
            (void)hipGetLastError();
            set_error("launch_cnn_fused: cannot raise the kernel's LDS limit");
            return FMGMC_EHIP;
        }
        attr_set = true;
    }
    FusedArgs f{};
    f.n = n;
    f.in0 = a.in0;
    f.in1 = a.in1;
    f.in_stride = a.in_stride;
    f.log0 = a.log0;
    f.rr = a.rr;
    f.y = a.y;
    f.e = a.e;
    f.active = a.active;
    for (int k = 0; k < kCnnLayers; ++k) {
        f.w[k] = static_cast<const bf8 *>(w.w[k]);
        f.bias[k] = w.b[k];
    }
    const dim3 grid((n + FV - 1) / FV, a.S);
    hipLaunchKernelGGL(k_cnn_fused, grid, dim3(512), fused_lds_bytes(), st, f);
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
