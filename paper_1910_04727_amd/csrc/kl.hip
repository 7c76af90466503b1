// Karhunen-Loeve synthesis of the log-permeability (Section 3.1 (2)) as a
// dense contraction over modes, on the matrix cores of gfx950:
//   g[s][c] = sum_m xi[s][m] * B[m][c],
//   B[m][c] = sqrt(lambda_m) phi_{a_m}(x_i) phi_{b_m}(y_j),  c = j n + i,
//   K = exp(g) at the cell lower-left corners (x_i, y_j) = (i/n, j/n).
// B is never stored in HBM: each workgroup builds the slice of it that its
// cells need in LDS from the 1-D eigenfunction tables. The epilogue applies exp
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
// modes per axis. The epilogue (exp) writes 16 fine values per lane per tile.
// The coarse levels of the pyramid: the four waves take their tiles in rounds
// of 64 adjacent columns; a round's level-1 cells (even row, even column: 32
// x 32 of them) are staged in LDS, and after the round's barrier the workgroup
// stores them as whole rows, 32 adjacent coarse cells per row and store
// instruction, and the deeper levels from the same block. (Stored from the
// lanes that own them, they were short partial-line runs over every level,
// which cost as much as the fine field's own stores.)
constexpr int SB = 64;
constexpr int TSTR = SB + 16;
constexpr int L1S = 33;  // row stride (doubles) of the staged 32 x 32 level-1 block

template <int AP>
__global__ __launch_bounds__(256) void k_kl_sep_f64(KLArgs A, int S) {
    constexpr int CSd = AP + 2;
    constexpr int KK = AP / 4;
    static_assert(CSd <= TSTR, "C_s must fit in the space of T");
    extern __shared__ double sm[];
    double *Cm = sm;                 // [AP][CSd]   C_s[a][b]
    double *Tt = sm;                 // [AP][TSTR]  T_s[a][j] of the band (replaces C_s)
    double *L1 = sm + AP * TSTR;     // [32][L1S]   level-1 cells of one round of tiles
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
    const bool pyr = A.nlev > 1;
    for (int i0 = 16 * w; i0 < n; i0 += 64) {  // the same trip count in every wave
        d4 acc[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) acc[g] = d4{0.0, 0.0, 0.0, 0.0};
        // (unrolled by three: by four the level-1 staging pushes the kernel past 128
        // registers, three waves per SIMD instead of four)
#pragma unroll 3
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
                // level-1 cell (row 8g + 2v + r0/2, column 8w + c0/2 of the round's block)
                if (pyr && even) L1[(8 * g + 2 * v + (r0 >> 1)) * L1S + 8 * w + (c0 >> 1)] = kv;
            }
        }
        if (!pyr) continue;
        __syncthreads();
        // the round's block: level-1 rows J1 = j0/2 + Jb, columns I1 = 32 rnd + Ib. Its
        // origin is a multiple of 32, so on level k (sh = k - 1 <= 5) it is the block of
        // side 32 >> sh at the origin >> sh, whose cell (Jb, Ib) is level-1 cell
        // (Jb, Ib) << sh; deeper, it holds the one cell at the origin >> sh if the
        // origin is a multiple of 2^sh. Each level takes its own threads, a row of the
        // block per group of lanes, so its stores are whole rows of the block
        const int J1b = j0 >> 1, I1b = (i0 - 16 * w) >> 1;
#pragma unroll 1
        for (int k = 1, sh = 0; k < A.nlev; ++k, ++sh) {
            const bool in = sh <= 5 || ((J1b | I1b) & ((1 << sh) - 1)) == 0;
            const int side = in ? (sh <= 5 ? 32 >> sh : 1) : 0, lg = sh <= 5 ? 5 - sh : 0, nl = n >> k;
            for (int e = t; e < side * side; e += 256) {
                const int Jb = e >> lg, Ib = e & (side - 1);
                const double kv = L1[(Jb << sh) * L1S + (Ib << sh)];
                const size_t o = size_t(s) * nl * nl + size_t((J1b >> sh) + Jb) * nl + (I1b >> sh) + Ib;
                if (A.K64[k]) A.K64[k][o] = kv;
                if (A.K32[k]) A.K32[k][o] = float(kv);
            }
        }
        __syncthreads();
    }
}

template <int AP>
size_t sep_lds() {
    // C_s ([AP][AP+2]) and T ([AP][TSTR]) share the first part; then the level-1 block
    return (size_t(AP) * TSTR + 32 * L1S) * sizeof(double);
}

// ------------------------------------------------------ dense, FP32 / BF16 inputs
// v_mfma_f32_16x16x4_f32 (FP32) and v_mfma_f32_16x16x32_bf16 (BF16), FP32
// accumulation. Both operands are kept in the order the matrix cores take
// them, in 16-byte lane slots. Slot kc of a group of 16 rows (samples) or
// columns (cells) gives lane l = r + 16 h (row or column r) the modes
//   BF16, one K-step of 32 modes:   32 kc + 8 h + e,  e < 8,
//   FP32, four K-steps of 4 modes:  16 kc + 4 e + h,  e < 4 (element e feeds K-step 4 kc + e),
// so that every operand fetch of a wave is one contiguous 1 KB read. Each
// operand is rounded once, from FP64 to the input type (to nearest, ties to
// even; for BF16 not through FP32, which could round twice). xi is
// converted into that order once per launch (k_kl_xcvt, zero-padded to whole
// 16-sample groups and to a multiple of 32 modes). The Phi slice of a
// workgroup's 64 cells is built once in LDS (sqrt(lambda_m) phi_a(x_i)
// phi_b(y_j) in FP64) and reused for every sample
// tile the workgroup owns, so the gathers and FP64 products behind it are paid
// once per cell and mode, not once per sample tile. The A operand (xi) is read
// straight from L2 ahead of its use. Eight waves take 32 samples x 64 cells
// each (two 16-sample groups x four 16-cell groups, 8 accumulators).
// After the contraction the pass writes 12 bytes per fine cell and sample
// (FP64 and FP32 fields) plus the pyramid, and is bound by those writes.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

template <typename T> struct Lp;
template <> struct Lp<float> {
    typedef f4 V;
    static constexpr int CM = 16;  // modes per slot
    __device__ static int mode(int h, int e) { return 4 * e + h; }
};
template <> struct Lp<__bf16> {
    typedef bf8 V;
    static constexpr int CM = 32;
    __device__ static int mode(int h, int e) { return 8 * h + e; }
};
constexpr int LP_WAVES = 8;              // waves per workgroup
constexpr int LP_TILE = 32 * LP_WAVES;   // samples per sample tile
constexpr int LP_SLOTS = 32;             // Phi slots held in LDS at once (32 x 4 KB)
constexpr int LP_MPAD = 32;              // modes padded to a multiple of this

int lp_chunks(int M, int prec) {
    const int mp = (M + LP_MPAD - 1) / LP_MPAD * LP_MPAD;
    return mp / (prec == FMGMC_KL_BF16 ? Lp<__bf16>::CM : Lp<float>::CM);
}

template <typename T>
__global__ __launch_bounds__(256) void k_kl_xcvt(const double *xi, int S, int M, int nch, typename Lp<T>::V *out) {
    constexpr int EPS = 16 / sizeof(T);
    const int64_t slot = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (slot >= int64_t((S + 15) / 16) * nch * 64) return;
    const int l = int(slot & 63), kc = int((slot >> 6) % nch);
    const int64_t s = 16 * ((slot >> 6) / nch) + (l & 15);
    typename Lp<T>::V v;
#pragma unroll
    for (int e = 0; e < EPS; ++e) {
        const int m = Lp<T>::CM * kc + Lp<T>::mode(l >> 4, e);
        v[e] = T((s < S && m < M) ? xi[s * M + m] : 0.0);
    }
    out[slot] = v;
}

__device__ __forceinline__ void lp_mma(f4 (&acc)[2][4], const f4 &a0, const f4 &a1, const f4 (&b)[4]) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            acc[0][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[e], b[q][e], acc[0][q], 0, 0, 0);
            acc[1][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[e], b[q][e], acc[1][q], 0, 0, 0);
        }
}
__device__ __forceinline__ void lp_mma(f4 (&acc)[2][4], const bf8 &a0, const bf8 &a1, const bf8 (&b)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        acc[0][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b[q], acc[0][q], 0, 0, 0);
        acc[1][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b[q], acc[1][q], 0, 0, 0);
    }
}

// epilogue for one (sample, cell c of pyramid level k, an nk x nk plane): K = exp(g)
// into the level's FP64 and FP32 planes
__device__ __forceinline__ void lp_store(const KLArgs &A, int S, int k, int nk, int s, int c, float g) {
    if (s >= S || c >= nk * nk) return;
    const float kf = __expf(g);
    const size_t o = size_t(s) * nk * nk + c;
    if (A.K64[k]) __builtin_nontemporal_store(double(kf), A.K64[k] + o);
    if (A.K32[k]) __builtin_nontemporal_store(kf, A.K32[k] + o);
}

// 64-cell tiles of pyramid level k (cells of the nk x nk plane, nk = n / 2^k)
__host__ __device__ __forceinline__ int lp_level_tiles(int n, int k) {
    const int nk = n >> k;
    return (nk * nk + 63) / 64;
}

// Workgroup: 64 consecutive cells c0 .. c0+63 of one pyramid level's plane, samples
// [blockIdx.y sg, +sg) in tiles of LP_TILE. Every level is contracted for its own
// cells (cell (I, J) of level k is the grid point (2^k I, 2^k J), so its column of
// Phi, and with it every bit of g, is that of the fine cell it injects), which
// makes every store of every level a run of contiguous cells.
// The A slots of a wave stream through a ring of PF registers, PF slots ahead of
// their use (three for BF16, whose K-step is a quarter of the FP32 one's
// matrix-core time; one for FP32).
template <typename T>
__global__ __launch_bounds__(64 * LP_WAVES) void k_kl_lp(KLArgs A, int S, int sg, int nch) {
    typedef typename Lp<T>::V V;
    constexpr int CM = Lp<T>::CM, EPS = 16 / sizeof(T), PF = sizeof(T) == 2 ? 3 : 1;
    extern __shared__ __align__(16) unsigned char lp_lds[];
    V *Bs = reinterpret_cast<V *>(lp_lds);  // [slot][16-cell group q][lane]
    const int n = A.n, M = A.M;
    int lev = 0, tile = blockIdx.x;
    while (lev + 1 < A.nlev && tile >= lp_level_tiles(n, lev)) tile -= lp_level_tiles(n, lev++);
    const int nk = n >> lev, c0 = tile * 64, sb = blockIdx.y * sg, se = min(S, sb + sg);
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const V *X = static_cast<const V *>(A.xw);
    // slice builder: thread t fills the slots of cell group bq, lane l, every other slot
    const int bq = w & 3, bh = w >> 2, bc = c0 + 16 * bq + (l & 15);
    const bool bval = bc < nk * nk;
    const int bi = bval ? (bc % nk) << lev : 0, bj = bval ? (bc / nk) << lev : 0;
    auto build = [&](int kb0, int nb) {
        for (int k = bh; k < nb; k += 2) {
            V v;
#pragma unroll
            for (int e = 0; e < EPS; ++e) {
                const int m = CM * (kb0 + k) + Lp<T>::mode(l >> 4, e);
                double b = 0.0;
                if (bval && m < M)
                    b = A.sqrtlam[m] * A.phi[size_t(A.ma[m]) * n + bi] * A.phi[size_t(A.mb[m]) * n + bj];
                v[e] = T(b);
            }
            Bs[(k * 4 + bq) * 64 + l] = v;
        }
    };
    const bool resident = nch <= LP_SLOTS;
    if (resident) {
        build(0, nch);
        __syncthreads();
    }
    const V zero = V{};
    for (int st = sb; st < se; st += LP_TILE) {
        const int s0 = st + 32 * w;
        const bool act = s0 < se, two = s0 + 16 < se;
        f4 acc[2][4];
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[r][q] = f4{0.f, 0.f, 0.f, 0.f};
        for (int kb0 = 0; kb0 < nch; kb0 += LP_SLOTS) {
            const int nb = min(LP_SLOTS, nch - kb0);
            if (!resident) {
                __syncthreads();
                build(kb0, nb);
                __syncthreads();
            }
            if (!act) continue;
            const V *x0 = X + (size_t(s0 / 16) * nch + kb0) * 64 + l;
            const V *x1 = x0 + size_t(nch) * 64;
            V r0[PF], r1[PF];
#pragma unroll
            for (int j = 0; j < PF; ++j) {
                r0[j] = j < nb ? x0[j * 64] : zero;
                r1[j] = (j < nb && two) ? x1[j * 64] : zero;
            }
            for (int k0 = 0; k0 < nb; k0 += PF) {
#pragma unroll
                for (int j = 0; j < PF; ++j) {
                    const int k = k0 + j;
                    if (k < nb) {
                        const V a0 = r0[j], a1 = r1[j];
                        if (k + PF < nb) {
                            r0[j] = x0[(k + PF) * 64];
                            if (two) r1[j] = x1[(k + PF) * 64];
                        }
                        V b[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) b[q] = Bs[(k * 4 + q) * 64 + l];
                        lp_mma(acc, a0, a1, b);
                    }
                }
            }
        }
        if (!act) continue;
        // lane l holds rows 4 (l/16) + v, column l%16 of each 16 x 16 output
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    lp_store(A, S, lev, nk, s0 + 16 * r + 4 * (l >> 4) + v, c0 + 16 * q + (l & 15), acc[r][q][v]);
    }
}

template <typename T>
int launch_lp(const KLArgs &a, int S, int prec, hipStream_t st) {
    typedef typename Lp<T>::V V;
    const int nch = lp_chunks(a.M, prec);
    const size_t lds = size_t(std::min(nch, LP_SLOTS)) * 4 * 64 * sizeof(V);
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(k_kl_lp<T>),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       int(size_t(LP_SLOTS) * 4 * 64 * sizeof(V)));
    if (attr != hipSuccess) {
        set_error("launch_kl: cannot raise the kernel's LDS limit");
        return FMGMC_EHIP;
    }
    const int64_t slots = int64_t((S + 15) / 16) * nch * 64;
    hipLaunchKernelGGL(k_kl_xcvt<T>, dim3(unsigned((slots + 255) / 256)), dim3(256), 0, st, a.xi, S, a.M, nch,
                       static_cast<V *>(a.xw));
    // enough workgroups to fill the chip; each keeps its Phi slice for as many
    // sample tiles as that allows
    int nct = 0;
    for (int k = 0; k < a.nlev; ++k) nct += lp_level_tiles(a.n, k);
    const int tiles = (S + LP_TILE - 1) / LP_TILE;
    const int groups = std::max(1, std::min(tiles, (1024 + nct - 1) / nct));
    const int sg = (tiles + groups - 1) / groups * LP_TILE;
    hipLaunchKernelGGL(k_kl_lp<T>, dim3(nct, (S + sg - 1) / sg), dim3(64 * LP_WAVES), lds, st, a, S, sg, nch);
    return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP;
}

}  // namespace

size_t kl_work_bytes(int S, int M, int prec) {
    if (prec != FMGMC_KL_FP32 && prec != FMGMC_KL_BF16) return 0;
    return size_t((S + 15) / 16) * lp_chunks(M, prec) * 64 * 16;
}

bool kl_separable(const KLArgs &a, int prec) {
    return prec == FMGMC_KL_FP64 && a.n >= SB && a.n % SB == 0 && a.kdim >= 1 && a.kdim <= 64;
}

double kl_flops(const KLArgs &a, int prec) {
    const double n = a.n, kd = a.kdim;
    if (kl_separable(a, prec)) return 2.0 * kd * n * (kd + n);
    double cells = double(n) * n;  // the FP32 / BF16 contraction also computes the coarse levels' cells
    if (prec == FMGMC_KL_FP32 || prec == FMGMC_KL_BF16)
        for (int k = 1; k < a.nlev; ++k) cells += double(a.n >> k) * (a.n >> k);
    return 2.0 * double(a.M) * cells;
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
    else if (prec == FMGMC_KL_FP32 || prec == FMGMC_KL_BF16) {
        if (!a.xw) {
            set_error("launch_kl: the FP32 / BF16 contraction needs its xi workspace");
            return FMGMC_EINVAL;
        }
        return prec == FMGMC_KL_FP32 ? launch_lp<float>(a, S, prec, st) : launch_lp<__bf16>(a, S, prec, st);
    } else {
        set_error("launch_kl: unknown precision");
        return FMGMC_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP;
}

}  // namespace fmgmc
