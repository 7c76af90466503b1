// Karhunen-Loeve synthesis of the log-permeability (Section 3.1 (2)) as a
// dense contraction over modes, on the matrix cores of gfx950:
//   g[s][c] = sum_m xi[s][m] * B[m][c],
//   B[m][c] = sqrt(lambda_m) phi_{a_m}(x_i) phi_{b_m}(y_j),  c = j n + i,
//   K = exp(g) at the cell lower-left corners (x_i, y_j) = (i/n, j/n).
// B is never stored in HBM: each workgroup builds its 64-mode x 64-cell slice
// of it in LDS from the 1-D eigenfunction tables. The epilogue applies exp
// and writes every level of the injected coefficient pyramid
// (Section 2.5, Coarsening): cell (i, j) of the fine grid also serves as cell
// (i/2^k, j/2^k) of level k whenever 2^k divides both i and j.
#include "common.h"

namespace fmgmc {

namespace {

constexpr int TS = 64;     // samples per tile
constexpr int TC = 64;     // cells per tile
constexpr int TM = 64;     // modes per LDS chunk
// LDS row strides (elements) chosen so that the MFMA operand reads hit
// distinct banks: A reads 16 rows x 4 k-columns, B reads 4 k-rows x 16
// columns. FP64 (8-byte reads, 32 lanes per pass): A stride = 2 mod 32
// doubles, B stride = 16 mod 32. FP32: A stride = 4 mod 64, B stride = 16 mod 64.
template <typename T> constexpr int xstr() { return sizeof(T) == 8 ? TM + 2 : TM + 4; }
constexpr int BSTR = TC + 16;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// epilogue shared by all precisions: value g for (sample, cell)
__device__ __forceinline__ void store_pyramid(const KLArgs &A, int S, int s, int c, double g, bool f32exp) {
    if (s >= S) return;
    const int n = A.n;
    if (c >= n * n) return;
    const int i = c % n, j = c / n;
    const double kv = f32exp ? double(__expf(float(g))) : exp(g);
    int nl = n, ii = i, jj = j;
    for (int k = 0; k < A.nlev; ++k) {
        const size_t o = size_t(s) * nl * nl + size_t(jj) * nl + ii;
        if (A.K64[k]) A.K64[k][o] = kv;
        if (A.K32[k]) A.K32[k][o] = float(kv);
        if ((ii & 1) || (jj & 1)) break;
        ii >>= 1;
        jj >>= 1;
        nl >>= 1;
    }
}

// Element e of the 64-mode x 64-cell slice Bt[m][c] (modes m0.., cells c0..):
// sqrt(lambda_m) phi_{a_m}(x_i) phi_{b_m}(y_j). When the cell tile lies in one
// grid row j (n >= TC), rowf[m] = sqrt(lambda_m) phi_{b_m}(y_j) and ia[m] = a_m n
// are staged in LDS once per workgroup.
__device__ __forceinline__ double b_elem(const KLArgs &A, int m0, int c0, int e, const double *rowf, const int *ia) {
    const int n = A.n, mm = e / TC, cc = e % TC, m = m0 + mm;
    if (m >= A.M) return 0.0;
    if (rowf) return rowf[m] * A.phi[ia[m] + (c0 % n) + cc];
    const int c = c0 + cc;
    if (c >= n * n) return 0.0;
    const int i = c % n, j = c / n;
    return A.sqrtlam[m] * A.phi[size_t(A.ma[m]) * n + i] * A.phi[size_t(A.mb[m]) * n + j];
}

// stages rowf / ia for a one-row tile; returns whether it applies
__device__ __forceinline__ bool stage_row(const KLArgs &A, int c0, double *rowf, int *ia) {
    const int n = A.n;
    if (n < TC) return false;
    const int j = c0 / n;
    for (int m = threadIdx.x; m < A.M; m += blockDim.x) {
        rowf[m] = A.sqrtlam[m] * A.phi[size_t(A.mb[m]) * n + j];
        ia[m] = A.ma[m] * n;
    }
    return true;
}

__device__ __forceinline__ double xi_elem(const KLArgs &A, int S, int s0, int m0, int e) {
    const int s = s0 + e / TM, m = m0 + e % TM;
    return (s < S && m < A.M) ? A.xi[size_t(s) * A.M + m] : 0.0;
}

// Both MFMA forms share the schedule: the A (xi) and B (Phi) values of chunk
// k + 1 are loaded into registers while the matrix cores work on chunk k from
// LDS, so global latency hides behind the contraction.
constexpr int PER = TS * TM / 256;  // elements per thread per chunk (both tiles are 64 x 64)

// FP64: v_mfma_f64_16x16x4_f64. Lane l: A[row l%16][k l/16], B[k l/16][col l%16];
// output register v of lane l holds row 4 v + l/16, column l%16 (one row per
// 16-lane group per register, unlike the FP32/BF16 16x16 forms).
__global__ __launch_bounds__(256) void k_kl_f64(KLArgs A, int S) {
    constexpr int XSTR = xstr<double>();
    __shared__ double Xs[TS * XSTR];
    __shared__ double Bt[TM * BSTR];
    extern __shared__ double rowf[];  // [M] then int ia[M]
    int *ia = reinterpret_cast<int *>(rowf + A.M);
    const int c0 = blockIdx.x * TC, s0 = blockIdx.y * TS;
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const bool row = stage_row(A, c0, rowf, ia);
    __syncthreads();
    const double *rf = row ? rowf : nullptr;
    double xr[PER], br[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        xr[k] = xi_elem(A, S, s0, 0, t + 256 * k);
        br[k] = b_elem(A, 0, c0, t + 256 * k, rf, ia);
    }
    d4 acc[4];
    for (int q = 0; q < 4; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
    for (int m0 = 0; m0 < A.M; m0 += TM) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = t + 256 * k;
            Xs[(e / TM) * XSTR + e % TM] = xr[k];
            Bt[(e / TC) * BSTR + e % TC] = br[k];
        }
        __syncthreads();
        if (m0 + TM < A.M) {
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                xr[k] = xi_elem(A, S, s0, m0 + TM, t + 256 * k);
                br[k] = b_elem(A, m0 + TM, c0, t + 256 * k, rf, ia);
            }
        }
#pragma unroll 4
        for (int kk = 0; kk < TM / 4; ++kk) {
            const double a = Xs[(16 * w + (l & 15)) * XSTR + 4 * kk + (l >> 4)];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double b = Bt[(4 * kk + (l >> 4)) * BSTR + 16 * q + (l & 15)];
                acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[q], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            store_pyramid(A, S, s0 + 16 * w + 4 * v + (l >> 4), c0 + 16 * q + (l & 15), acc[q][v], false);
}

// FP32: v_mfma_f32_16x16x4_f32, same operand layout as the FP64 form; output
// register v of lane l holds row 4 (l/16) + v, column l%16.
__global__ __launch_bounds__(256) void k_kl_f32(KLArgs A, int S) {
    constexpr int XSTR = xstr<float>();
    __shared__ float Xs[TS * XSTR];
    __shared__ float Bt[TM * BSTR];
    extern __shared__ double rowf[];  // [M] then int ia[M]
    int *ia = reinterpret_cast<int *>(rowf + A.M);
    const int c0 = blockIdx.x * TC, s0 = blockIdx.y * TS;
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const bool row = stage_row(A, c0, rowf, ia);
    __syncthreads();
    const double *rf = row ? rowf : nullptr;
    float xr[PER], br[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        xr[k] = float(xi_elem(A, S, s0, 0, t + 256 * k));
        br[k] = float(b_elem(A, 0, c0, t + 256 * k, rf, ia));
    }
    f4 acc[4];
    for (int q = 0; q < 4; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
    for (int m0 = 0; m0 < A.M; m0 += TM) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = t + 256 * k;
            Xs[(e / TM) * XSTR + e % TM] = xr[k];
            Bt[(e / TC) * BSTR + e % TC] = br[k];
        }
        __syncthreads();
        if (m0 + TM < A.M) {
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                xr[k] = float(xi_elem(A, S, s0, m0 + TM, t + 256 * k));
                br[k] = float(b_elem(A, m0 + TM, c0, t + 256 * k, rf, ia));
            }
        }
#pragma unroll 4
        for (int kk = 0; kk < TM / 4; ++kk) {
            const float a = Xs[(16 * w + (l & 15)) * XSTR + 4 * kk + (l >> 4)];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float b = Bt[(4 * kk + (l >> 4)) * BSTR + 16 * q + (l & 15)];
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[q], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            store_pyramid(A, S, s0 + 16 * w + 4 * (l >> 4) + v, c0 + 16 * q + (l & 15), double(acc[q][v]), true);
}

// ---------------------------------------------------------------- separable
// For the separable covariance every 2-D mode is a product of 1-D modes
// (Section 3.1 (2)), so the same sum factors through a small per-sample matrix:
//   g_s(x_i, y_j) = sum_a phi_a(x_i) T_s[a][j],   T_s[a][j] = sum_b C_s[a][b] phi_b(y_j),
//   C_s[a_m][b_m] = xi_s[m] sqrt(lambda_m), zero for pairs that are not kept modes.
// With A 1-D modes per axis (A <= 64) this is 2 (A + n) A n flops per sample
// instead of 2 M n^2, and the pass is bound by writing the coefficient pyramid.
// Workgroup: one sample and a band of 64 grid rows; T for the band is formed
// once (FP64 MFMA). Then each wave takes its own 16-column x-tiles (every 4th)
// over all 64 rows: g[j][i] = sum_a T[a][j] phi_a(x_i), four 16 x 16 FP64 MFMA
// outputs per tile, A operands (T) from LDS, B operands phi_a(x_i) from the
// L2-resident [kdim][n] table; no two waves load the same operand, and no
// barrier separates the tiles. LDS holds only C_s, then T
// (the same space, 80-double rows, conflict-free operand reads): 30 KB at 48
// modes per axis. The epilogue (exp, the pyramid) writes 16 values per lane
// per tile; the parity of a lane's rows and columns is fixed, so the coarse
// levels are taken only by the lanes that own even cells.
constexpr int SB = 64;
constexpr int TSTR = SB + 16;

// levels >= 1 of the pyramid for one fine cell (i, j) with both indices even
__device__ __forceinline__ void store_coarse(const KLArgs &A, int s, int i, int j, double kv) {
    int nl = A.n, ii = i, jj = j;
    for (int k = 1; k < A.nlev; ++k) {
        ii >>= 1;
        jj >>= 1;
        nl >>= 1;
        const size_t o = size_t(s) * nl * nl + size_t(jj) * nl + ii;
        if (A.K64[k]) A.K64[k][o] = kv;
        if (A.K32[k]) A.K32[k][o] = float(kv);
        if ((ii & 1) || (jj & 1)) break;
    }
}

template <int AP>
__global__ __launch_bounds__(256) void k_kl_sep_f64(KLArgs A, int S) {
    constexpr int CSd = AP + 2;
    constexpr int KK = AP / 4;
    static_assert(CSd <= TSTR, "C_s must fit in the space of T");
    extern __shared__ double sm[];
    double *Cm = sm;                 // [AP][CSd]   C_s[a][b]
    double *Tt = sm;                 // [AP][TSTR]  T_s[a][j] of the band (replaces C_s)
    const int n = A.n, s = blockIdx.y, j0 = blockIdx.x * SB, KD = A.kdim;
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    if (s >= S) return;
    for (int e = t; e < AP * CSd; e += 256) Cm[e] = 0.0;
    __syncthreads();
    for (int m = t; m < A.M; m += 256) Cm[A.ma[m] * CSd + A.mb[m]] = A.xi[size_t(s) * A.M + m] * A.sqrtlam[m];
    __syncthreads();
    // phi_k(s_i) for k < KD (zero for the padding modes k >= KD)
    auto phi = [&](int k, int i) -> double { return k < KD ? A.phi[size_t(k) * n + i] : 0.0; };
    {   // T[a][j] = sum_b C[a][b] phi_b(y_j): wave w owns the j columns 16w .. 16w+15
        d4 acc[AP / 16];
#pragma unroll
        for (int q = 0; q < AP / 16; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int kk = 0; kk < KK; ++kk) {
            const double bv = phi(4 * kk + (l >> 4), j0 + 16 * w + (l & 15));
#pragma unroll
            for (int q = 0; q < AP / 16; ++q) {
                const double av = Cm[(16 * q + (l & 15)) * CSd + 4 * kk + (l >> 4)];
                acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[q], 0, 0, 0);
            }
        }
        __syncthreads();  // every wave's reads of C_s are done before T overwrites it
#pragma unroll
        for (int q = 0; q < AP / 16; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v) Tt[(16 * q + 4 * v + (l >> 4)) * TSTR + 16 * w + (l & 15)] = acc[q][v];
    }
    __syncthreads();
    // lane l holds output rows 4v + l/16 (+16g) and column l%16 of a tile
    const int r0 = l >> 4, c0 = l & 15;
    const bool even = ((r0 | c0) & 1) == 0;
    for (int i0 = 16 * w; i0 < n; i0 += 64) {
        d4 acc[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) acc[g] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int kk = 0; kk < KK; ++kk) {
            const double bv = phi(4 * kk + r0, i0 + c0);
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const double av = Tt[(4 * kk + r0) * TSTR + 16 * g + c0];
                acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[g], 0, 0, 0);
            }
        }
        const int i = i0 + c0;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
#pragma unroll 1
            for (int v = 0; v < 4; ++v) {
                const int j = j0 + 16 * g + 4 * v + r0;
                const double kv = exp(acc[g][v]);
                const size_t o = size_t(s) * n * n + size_t(j) * n + i;
                // the fine field streams out (read back only by later passes)
                if (A.K64[0]) __builtin_nontemporal_store(kv, A.K64[0] + o);
                if (A.K32[0]) __builtin_nontemporal_store(float(kv), A.K32[0] + o);
                if (even) store_coarse(A, s, i, j, kv);
            }
        }
    }
}

template <int AP>
size_t sep_lds() {
    return size_t(AP) * TSTR * sizeof(double);  // C_s ([AP][AP+2]) and T ([AP][TSTR]) share it
}

// BF16 inputs, FP32 accumulation: v_mfma_f32_16x16x32_bf16. Lane l holds
// A[row l%16][k = 8 (l/16) .. +7] and B[k = 8 (l/16) .. +7][col l%16]; D as above.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__global__ __launch_bounds__(256) void k_kl_bf16(KLArgs A, int S) {
    __shared__ __bf16 Xs[TS * (TM + 8)];
    __shared__ __bf16 Bt[TC * (TM + 8)];   // transposed: [cell][mode]
    const int c0 = blockIdx.x * TC, s0 = blockIdx.y * TS;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    f4 acc[4];
    for (int q = 0; q < 4; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
    const int n = A.n;
    for (int m0 = 0; m0 < A.M; m0 += TM) {
        __syncthreads();
        for (int e = threadIdx.x; e < TS * TM; e += blockDim.x) {
            const int ss = e / TM, mm = e % TM, s = s0 + ss, m = m0 + mm;
            const double v = (s < S && m < A.M) ? A.xi[size_t(s) * A.M + m] : 0.0;
            Xs[ss * (TM + 8) + mm] = __bf16(float(v));
        }
        for (int e = threadIdx.x; e < TM * TC; e += blockDim.x) {
            const int mm = e / TC, cc = e % TC, m = m0 + mm, c = c0 + cc;
            double v = 0.0;
            if (m < A.M && c < n * n)
                v = A.sqrtlam[m] * A.phi[size_t(A.ma[m]) * n + (c % n)] * A.phi[size_t(A.mb[m]) * n + (c / n)];
            Bt[cc * (TM + 8) + mm] = __bf16(float(v));
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TM / 32; ++kk) {
            bf8 a, b;
            const __bf16 *pa = Xs + (16 * w + (l & 15)) * (TM + 8) + 32 * kk + 8 * (l >> 4);
#pragma unroll
            for (int e = 0; e < 8; ++e) a[e] = pa[e];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const __bf16 *pb = Bt + (16 * q + (l & 15)) * (TM + 8) + 32 * kk + 8 * (l >> 4);
#pragma unroll
                for (int e = 0; e < 8; ++e) b[e] = pb[e];
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[q], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            store_pyramid(A, S, s0 + 16 * w + 4 * (l >> 4) + v, c0 + 16 * q + (l & 15), double(acc[q][v]), true);
}

}  // namespace

bool kl_separable(const KLArgs &a, int prec) {
    return prec == FMGMC_KL_FP64 && a.n >= SB && a.n % SB == 0 && a.kdim >= 1 && a.kdim <= 64;
}

double kl_flops(const KLArgs &a, int prec) {
    const double n = a.n, kd = a.kdim;
    return kl_separable(a, prec) ? 2.0 * kd * n * (kd + n) : 2.0 * double(a.M) * n * n;
}

int launch_kl(const KLArgs &a, int S, int prec, hipStream_t st) {
    if (S <= 0) return FMGMC_OK;
    if (kl_separable(a, prec)) {
        const dim3 g(a.n / SB, S), b(256);
        const int ap = (a.kdim + 15) / 16 * 16;
        if (ap == 16) hipLaunchKernelGGL(k_kl_sep_f64<16>, g, b, sep_lds<16>(), st, a, S);
        else if (ap == 32) hipLaunchKernelGGL(k_kl_sep_f64<32>, g, b, sep_lds<32>(), st, a, S);
        else if (ap == 48) hipLaunchKernelGGL(k_kl_sep_f64<48>, g, b, sep_lds<48>(), st, a, S);
        else hipLaunchKernelGGL(k_kl_sep_f64<64>, g, b, sep_lds<64>(), st, a, S);
        return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP;
    }
    dim3 grid((a.n * a.n + TC - 1) / TC, (S + TS - 1) / TS), block(256);
    const size_t dyn = size_t(a.M) * (sizeof(double) + sizeof(int));
    if (prec == FMGMC_KL_FP64 || prec == FMGMC_KL_FP64_DENSE) hipLaunchKernelGGL(k_kl_f64, grid, block, dyn, st, a, S);
    else if (prec == FMGMC_KL_FP32) hipLaunchKernelGGL(k_kl_f32, grid, block, dyn, st, a, S);
    else if (prec == FMGMC_KL_BF16) hipLaunchKernelGGL(k_kl_bf16, grid, block, 0, st, a, S);
    else {
        set_error("launch_kl: unknown precision");
        return FMGMC_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP;
}

}  // namespace fmgmc
