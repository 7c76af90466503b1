// Fused red-black Gauss-Seidel passes for the cell-centred five-point
// finite-volume operator (Section 3.1 (1)), used by the V-cycles of the full
// multigrid pass (Section 2.5).
//
// Design (gfx950): one workgroup owns one sample; lane l owns the two cells
// of columns 2l and 2l+1 of every row, one red and one black, so every lane
// updates exactly one cell in every half-sweep. The workgroup marches up the
// rows. At step F it takes row F (loaded NH+1 steps earlier into a register
// queue, three in the FP32 passes of eight half-sweeps, so HBM latency
// overlaps the work of that many rows) and applies half-sweep t (t = 1..NH,
// red first) to row F - t: this is the wavefront order of the
// sweeps, so the result is exactly that of NH sequential half-sweeps. The
// residual follows at row F - NH - 1 and is summed over 2x2 blocks into the
// next coarser grid and/or squared into the sample's residual norm. Every
// cell is read and written once per pass.
// The pre-smoothing pass of an FP32 cycle that follows an FP64 refinement can
// take the refinement itself (INIT_IR): the residual of each row, formed in
// FP64 one row ahead of the sweeps, is that row's right-hand side.
// Rows in flight live in an LDS ring padded with a zero column on each side,
// and the ring rows below row 0 and above row n-1 read as zero when those rows
// are swept, so boundary neighbours contribute nothing without a branch (a
// boundary face enters only the diagonal and the right-hand side); per-row
// coefficients live in a register ring. One barrier per row step: every
// cross-lane read in step F is of data written before step F's barrier.
// Boundary conditions: Case II (Dirichlet west/east, no flow south/north) or
// Case I (Dirichlet on all sides) of Table 1, a uniform runtime switch.
#include <type_traits>

#include "common.h"

namespace fmgmc {

template <typename T>
struct V2 {
    T a, b;
};

template <typename T>
__device__ __forceinline__ T harm(T a, T b) {
    return T(2) * a * b * rcp_(a + b);
}

// c ? a : b with both operands evaluated on every lane: the compiler otherwise
// guards the costlier one (a neighbour's load, a harmonic mean) by an
// exec-mask branch, for the single lane at a side of the grid
template <typename T>
__device__ __forceinline__ T lane_sel(bool c, T a, T b) {
    if constexpr (sizeof(T) == 4) {
        const uint32_t m = 0u - uint32_t(c);
        return __builtin_bit_cast(T, (__builtin_bit_cast(uint32_t, a) & m) | (__builtin_bit_cast(uint32_t, b) & ~m));
    } else {
        const uint64_t m = 0ull - uint64_t(c);
        return __builtin_bit_cast(T, (__builtin_bit_cast(uint64_t, a) & m) | (__builtin_bit_cast(uint64_t, b) & ~m));
    }
}

template <typename T>
__device__ __forceinline__ V2<T> ld2(const T *p) {
    if constexpr (sizeof(T) == 8) {
        const double2 v = *reinterpret_cast<const double2 *>(p);
        return {T(v.x), T(v.y)};
    } else {
        const float2 v = *reinterpret_cast<const float2 *>(p);
        return {T(v.x), T(v.y)};
    }
}

template <typename T>
__device__ __forceinline__ void st2(T *p, T a, T b) {
    if constexpr (sizeof(T) == 8) {
        *reinterpret_cast<double2 *>(p) = double2{a, b};
    } else {
        *reinterpret_cast<float2 *>(p) = float2{a, b};
    }
}

// streamed operands (each read or written once per pass, so caching them only
// displaces data that is reused): non-temporal 2-cell loads and stores
template <typename T>
__device__ __forceinline__ V2<T> ld2_nt(const T *p) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(p));
    return {v.x, v.y};
}

template <typename T>
__device__ __forceinline__ void st2_nt(T *p, T a, T b) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store(v2{a, b}, reinterpret_cast<v2 *>(p));
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, T *red) {
    // butterfly over the wave's lanes of this workgroup (fewer than 64 for n < 128)
    for (int o = min(32, int(blockDim.x) >> 1); o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    T t = 0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int k = 0; k < nw; ++k) t += red[k];
    }
    return t;
}

// rows of x alive at one step: the row being loaded, the NH rows being swept,
// their lower neighbour and the row whose residual is formed
constexpr int march_ring_rows(int nh) { return nh + 3 <= 8 ? 8 : 16; }

// minimum waves per SIMD the register allocation must allow: three for the
// refinement start with the interpolated iterate (167 VGPRs and 36 B per lane
// spilled; left alone the compiler takes 173 VGPRs, two waves per SIMD, and
// the pass measured 12% slower at 512^2)
template <int INIT, int OUT>
constexpr int march_min_waves() { return (INIT == INIT_IR && (OUT & OUT_PINTERP)) ? 3 : 1; }

template <typename T, int NH, bool CK, int INIT, bool RHSA, int OUT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(march_min_waves<INIT, OUT>())))
void k_march(MarchArgs<T> A) {
    constexpr int U = NH + 1;    // register ring depth = unroll
    constexpr int RX = march_ring_rows(NH);  // LDS x ring rows (>= NH + 3), power of two
    // prefetch distance of the load queue (a divisor of U, so that a row's queue
    // slot is a constant after unrolling, and row F + D lands in the slot that
    // step F + D reads): U rows; three in the FP32 stage-grid passes of eight
    // half-sweeps, whose registers then fit three waves per SIMD (see RC
    // below; 7% faster so); one in the correction passes (coefficients from
    // faces, grids below the stage grid) and in the FP64 post-smoothing passes
    // of the stage operator, whose row steps are long enough to cover a load.
    // The registers that frees (FP32 with RI below: 145-152 -> 99-109 VGPRs;
    // FP64 correction passes: 244-256 with a spill -> 186-194 without) take the
    // FP32 passes to four waves per SIMD, so that all 4096 one-wave workgroups
    // of a 128^2 or 64^2 pass are resident at once (FP32+IR +1.3-2.7%, FP64
    // form +1.8%, same-box A/B), and let the FP64 post-smoothing pass run
    // straight-line steps (see the row loops).
    constexpr int D = !CK ? 1 : (sizeof(T) == 4 && U % 3 == 0 && NH >= 6) ? 3
                    : (sizeof(T) == 8 && INIT == INIT_PROLONG) ? 1 : U;
    static_assert(U % D == 0, "the load queue depth must divide the unroll");
    constexpr bool RES = (OUT & (OUT_RESTRICT | OUT_RR)) != 0;
    constexpr bool CO = (INIT == INIT_PROLONG || INIT == INIT_INTERP);
    constexpr bool LX = (INIT == INIT_LOAD || INIT == INIT_PROLONG);
    // INIT_IR: the FP64 refinement of the stage iterate runs one row ahead of the
    // sweeps. At step F row F + 1 of p (+ e) and K64 enters their LDS rings; after
    // the step's barrier the residual of row F is formed in FP64 and, rounded to
    // FP32, is row F's right-hand side (and K of row F is float(K64))
    constexpr bool IR = (INIT == INIT_IR);
    constexpr bool PU = IR && (OUT & OUT_PUPD) != 0;
    static_assert(!IR || (sizeof(T) == 4 && CK && RHSA && (OUT & ~(OUT_PUPD | OUT_FACES | OUT_PINTERP)) == OUT_RESTRICT),
                  "the refinement start is an FP32 pre-smoothing pass of the stage operator");
    // OUT_FACES: coarse faces written as the coefficients of each odd row are formed
    constexpr bool FO = (OUT & OUT_FACES) != 0;
    static_assert(!FO || (IR && !(OUT & OUT_PUPD)) || (CK && INIT == INIT_INTERP && !RHSA),
                  "faces are written by the top stage's first pass");
    // OUT_PINTERP: row F + 1 of p formed at step F from a 4-row LDS ring of coarse
    // rows (slot = row & 3; the ghost rows -1 and n/2 in slots 3 and (n/2) & 3):
    // coarse row (F + 3) / 2 enters at odd steps F (rows 0 and 1 before the
    // first), so that the rows a step reads were written before its barrier and
    // the row it writes is none of them
    constexpr bool PI = (OUT & OUT_PINTERP) != 0;
    static_assert(!PI || FO, "the interpolated start is the top stage's first refinement");
    const int n = A.n, nl = n >> 1, nc = n >> 1;
    const int l = threadIdx.x;
    const int s = blockIdx.x;
    if (A.active && A.active[s] == 0) return;  // uniform over the block

    extern __shared__ unsigned char smem_raw[];
    const int XS = n + 4;                               // x row: [pad, pad, cells 0..n-1, pad, pad]
    T *xs = reinterpret_cast<T *>(smem_raw);            // [RX][XS]
    T *ks = xs + RX * XS;                               // [4][n] K (stage) or west faces (correction)
    T *cs = ks + 4 * n;                                 // [4][nc] coarse rows (prolongation source)
    T *red = cs + 4 * nc;                               // [16]
    // INIT_IR (in place of ks, cs and red, which it does not use)
    double *ks64 = reinterpret_cast<double *>(xs + RX * XS);  // [4][n] K64 rows
    double *ps64 = ks64 + 4 * n;                             // [3][n] rows of p (+ e)
    double *red64 = ps64 + 3 * n;                            // [18]
    double *cs64 = red64 + 18;                               // [4][n/2] coarse rows (PI)
    const size_t base = size_t(s) * n * n;
    // coarse row J of the solution on n/2 as it enters the ring: the ghost row
    // n/2 is the mirror of row n/2 - 1 (no flow) or 2 g - it (Dirichlet, Case I)
    const double *pcs = PI ? A.pc + size_t(s) * nc * nc : nullptr;
    auto cload = [&](int J) -> double { return pcs[size_t(min(J, nc - 1)) * nc + l]; };
    auto cput = [&](int J, double v) {
        cs64[(J & 3) * nc + l] = (J == nc && A.g.all) ? 2.0 * A.g.n - v : v;
    };
    double qcd = 0.0;  // PI: the coarse value of the next row to enter
    if constexpr (PI) {
        const double v0 = cload(0), v1 = cload(1);
        cput(0, v0);
        cput(1, v1);
        cs64[3 * nc + l] = A.g.all ? 2.0 * A.g.s - v0 : v0;  // ghost row -1
        qcd = cload(2);
    }
    for (int k = l; k < RX * XS; k += blockDim.x) xs[k] = T(0);
    __syncthreads();

    const size_t cbase = size_t(s) * nc * nc;
    const T gW = T(A.g.w), gE = T(A.g.e), gS = T(A.g.s), gN = T(A.g.n);
    const bool dns = A.g.all != 0;  // Dirichlet south / north sides (Case I)
    const T cgW = (INIT == INIT_INTERP) ? gW : T(0), cgE = (INIT == INIT_INTERP) ? gE : T(0);
    const T cgS = (INIT == INIT_INTERP) ? gS : T(0), cgN = (INIT == INIT_INTERP) ? gN : T(0);
    const bool first = (l == 0), last = (l == nl - 1);

    // prefetch queue, slot = row % D
    V2<T> qx[D], qk[D], qb[D], qf[D];
    T qc[D], qe[D];
    auto fetch = [&](int slot, int row) {
        const size_t idx = base + size_t(row) * n + 2 * l;
        if (LX) qx[slot] = ld2_nt(A.x + idx);
        if (CK) {
            qk[slot] = ld2_nt(A.K + idx);
        } else {
            qk[slot] = ld2_nt(A.f.fx + idx);
            qf[slot] = ld2_nt(A.f.fy + idx);
            qe[slot] = A.f.fxe[size_t(s) * n + row];
        }
        if (RHSA) qb[slot] = ld2_nt(A.b + idx);
        if (CO) {
            const int J = min((row + 1) >> 1, nc - 1);
            qc[slot] = A.xc[cbase + size_t(J) * nc + l];
        }
    };
    // INIT_IR: the next row of p, e and K64 in flight (one row: the unroll's five
    // rows in flight took 209 VGPRs, two waves per SIMD, and measured 2.6% slower
    // than this at three), held as vector types (the compiler kept the pair
    // struct in scratch memory here)
    typedef double d2v __attribute__((ext_vector_type(2)));
    typedef float f2v __attribute__((ext_vector_type(2)));
    d2v qp{0.0, 0.0}, qk64{0.0, 0.0};
    f2v qe2{0.0f, 0.0f};
    auto fetch_ir = [&](int row) __attribute__((always_inline)) {
        if constexpr (IR) {
            const size_t idx = base + size_t(row) * n + 2 * l;
            if constexpr (!PI) qp = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(A.p + idx));
            if constexpr (PU) qe2 = __builtin_nontemporal_load(reinterpret_cast<const f2v *>(A.e + idx));
            qk64 = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(A.K64 + idx));
        }
    };
    if constexpr (IR) {
        fetch_ir(0);
    } else {
#pragma unroll
        for (int u = 0; u < D; ++u)
            if (u < n) fetch(u, u);
    }
    // INIT_IR state: this lane's pairs of p (+ e) of the rows below / at / above
    // the residual's row, K64 of the residual's row and the one above, the north
    // faces of the row below (south faces of the residual's row), ||r||^2 and Q
    V2<double> pdn{0.0, 0.0}, pmid{0.0, 0.0}, pup{0.0, 0.0}, kmid{0.0, 0.0}, kup{0.0, 0.0}, tnp{0.0, 0.0};
    double rr64 = 0.0, q64 = 0.0;
    // PI: fine row R of p, the FMG interpolation of the ring's coarse rows R/2 and
    // the neighbour on R's side (ghosts at the boundary, as k_interp64 forms
    // them), written as the stage's start
    auto pinterp = [&](int R) -> V2<double> {
        const int J0 = R >> 1, J1 = J0 + ((R & 1) ? 1 : -1);
        const double *c0 = cs64 + (J0 & 3) * nc, *c1 = cs64 + (J1 & 3) * nc;
        const double a0 = c0[l], a1 = c1[l];
        const double w0 = lane_sel(first, 2.0 * A.g.w - a0, c0[max(l - 1, 0)]);
        const double w1 = lane_sel(first, 2.0 * A.g.w - a1, c1[max(l - 1, 0)]);
        const double e0 = lane_sel(last, 2.0 * A.g.e - a0, c0[min(l + 1, nc - 1)]);
        const double e1 = lane_sel(last, 2.0 * A.g.e - a1, c1[min(l + 1, nc - 1)]);
        const double p0 = (9.0 * a0 + 3.0 * w0 + 3.0 * a1 + w1) / 16.0;
        const double p1 = (9.0 * a0 + 3.0 * e0 + 3.0 * a1 + e1) / 16.0;
        st2_nt(A.p + base + size_t(R) * n + 2 * l, p0, p1);
        return V2<double>{p0, p1};
    };
    if constexpr (IR) {  // row 0 enters
        V2<double> pv{qp.x, qp.y};
        if constexpr (PI) pv = pinterp(0);
        if constexpr (PU) {
            pv.a += double(qe2.x);
            pv.b += double(qe2.y);
        }
        pmid = pv;
        kmid = V2<double>{qk64.x, qk64.y};
        st2(ps64 + 2 * l, pv.a, pv.b);
        st2(ks64 + 2 * l, kmid.a, kmid.b);
        fetch_ir(1);
    }

    // coefficient ring, slot = row % U: faces west of cell 0, between the cells,
    // east of cell 1; north faces and 1/diagonal of both cells; rhs (RHSA; a
    // boundary-data rhs is formed from the faces where it is used). No south-face
    // ring: a row's south faces are read as the north faces of the row below
    // (the same values). In FP64 that took the stage operator's post-smoothing
    // pass from a 100 B to a 52 B spill per lane and 8% off its time (FP64 form
    // +3%, bitwise unchanged, same-box A/B).
    T rw[U], rm[U], re[U], rn0[U], rn1[U], ri0[U], ri1[U], rb0[U], rb1[U];
#pragma unroll
    for (int k = 0; k < U; ++k)
        rw[k] = rm[k] = re[k] = rn0[k] = rn1[k] = ri0[k] = ri1[k] = rb0[k] = rb1[k] = T(0);
    V2<T> kprev{T(0), T(0)}, kcur{T(0), T(0)};   // own K (or south faces) of rows F-1, F
    V2<T> bprev{T(0), T(0)}, bcur{T(0), T(0)};
    T eprev = T(0), ecur = T(0);                 // east boundary face of rows F-1, F (correction)
    T rprev = T(0), rr = T(0), q = T(0);
    // FP32 passes of up to four half-sweeps, the FP64 stage-operator passes
    // with boundary-data right-hand sides and the FP64 correction passes: this
    // lane's cell pairs of the rows in flight (hv[t], the row that half-sweep t
    // acted on last; hv[0], the row that entered last; hres, the row below the
    // residual's row), so that the sweeps read only the west / east neighbours
    // from LDS. In FP64 that halves the LDS traffic that bounds these passes (two
    // waves per SIMD either way: 58 KB of LDS per 512^2 stage-operator workgroup
    // leave room for two per CU; 218-238 VGPRs for the correction passes, which
    // fit it without a spill since their load queue holds one row: +0.7%,
    // bitwise unchanged). The other passes read them from the LDS ring: their register
    // rings leave no room (the FP32 eight-half-sweep pass drops from 252 VGPRs,
    // two waves per SIMD, to 162, three; the refinement start, whose FP64 state
    // takes the room, keeps three waves per SIMD so, at 156-163 VGPRs).
    constexpr bool RC = (sizeof(T) == 4 && NH < 6 && !IR) || (sizeof(T) == 8 && (!CK || !RHSA));
    // FP64, the long FP32 passes, the refinement start and the correction
    // passes: 1/diagonal recomputed in each half-sweep from the coefficient ring
    // instead of being held in a ring of its own (registers, see D above)
    constexpr bool RI = sizeof(T) == 8 || NH >= 6 || IR || !CK;
    V2<T> hv[NH + 1];
#pragma unroll
    for (int t = 0; t <= NH; ++t) hv[t] = V2<T>{T(0), T(0)};
    V2<T> hres{T(0), T(0)};

    const int LAST = n - 1 + NH + (RES ? 1 : 0);
    // Row steps (march_step.inc). FP32: range-checked steps at both ends and
    // straight-line steps in between, so the prefetches of the queue are never
    // conditional and no wait for outstanding loads is forced at a merge; the
    // step is a lambda there (that keeps these kernels within 128 registers).
    // FP64: the step inline in the loops (behind a lambda the compiler kept one
    // of its queues in scratch memory), with the same checked and straight-line
    // steps. The stage operator's post-smoothing pass spills 100 B per lane so
    // (256 VGPRs, two waves per SIMD as before, which its LDS sets at 512^2) and
    // still takes 10% less time than with checked steps throughout (FP64 form
    // +4%); the correction passes (198-206 VGPRs, no spill) gave another +2.4%
    // (bitwise unchanged, same-box A/B).
    if constexpr (sizeof(T) == 4) {
        auto step = [&](const int F, const int u, auto chk) __attribute__((always_inline)) {
            constexpr bool C = decltype(chk)::value;
#include "march_step.inc"
        };
        const int lo = ((NH + 1 + U - 1) / U) * U;       // first unchecked step
        // first checked step after them
        const int hi = max(lo, ((n - U) / U) * U);
        int F0 = 0;
        for (; F0 < lo; F0 += U) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (F0 + u <= LAST) step(F0 + u, u, std::true_type{});
        }
        for (; F0 < hi; F0 += U) {
#pragma unroll
            for (int u = 0; u < U; ++u) step(F0 + u, u, std::false_type{});
        }
        for (; F0 <= LAST; F0 += U) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (F0 + u <= LAST) step(F0 + u, u, std::true_type{});
        }
    } else {
        const int lo = ((NH + 1 + U - 1) / U) * U;
        const int hi = max(lo, ((n - U) / U) * U);
        int F0 = 0;
        for (; F0 < lo; F0 += U) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int F = F0 + u;
                if (F > LAST) break;
                constexpr bool C = true;
#include "march_step.inc"
            }
        }
        for (; F0 < hi; F0 += U) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int F = F0 + u;
                constexpr bool C = false;
#include "march_step.inc"
            }
        }
        for (; F0 <= LAST; F0 += U) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int F = F0 + u;
                if (F > LAST) break;
                constexpr bool C = true;
#include "march_step.inc"
            }
        }
    }
    if constexpr (IR) {
        const double t = block_sum(rr64, red64);
        if (threadIdx.x == 0) A.rr[s] = t;
        if (!dns) {
            if (last) A.q[s] = q64;
        } else {
            if (l == (n >> 2) - 1) red64[16] = q64;
            if (l == (n >> 2)) red64[17] = q64;
            __syncthreads();
            if (l == 0) A.q[s] = (red64[16] + red64[17]) * 0.25;
        }
    }
    if (OUT & OUT_RR) {
        const T t = block_sum(rr, red);
        if (threadIdx.x == 0) A.rr[s] = double(t);
    }
    if (OUT & OUT_Q) {
        if (!dns) {
            if (last) A.q[s] = double(q);
        } else {
            // red[8], red[9] are not used by the residual reduction (at most 8 waves)
            if (l == (n >> 2) - 1) red[8] = q;
            if (l == (n >> 2)) red[9] = q;
            __syncthreads();
            if (l == 0) A.q[s] = double((red[8] + red[9]) * T(0.25));
        }
    }
}

// ------------------------------------------------------------------ dispatch
template <typename T, int NH>
static int dispatch_march(const MarchArgs<T> &a, int S, bool ck, int init, bool rhsa, int out,
                          hipStream_t st) {
    const int n = a.n;
    const size_t lds =
        init == INIT_IR
            ? size_t(march_ring_rows(NH)) * (n + 4) * sizeof(T) +
                  (7 * size_t(n) + 18 + ((out & OUT_PINTERP) ? 2 * size_t(n) : 0)) * sizeof(double)
            : (size_t(march_ring_rows(NH)) * (n + 4) + 4 * size_t(n) + 4 * size_t(n / 2) + 16) * sizeof(T);
    dim3 grid(S), block(n / 2);
#define FMGMC_MARCH_CASE(CKV, INITV, RHSV, OUTV)                                               \
    if (ck == CKV && init == INITV && rhsa == RHSV && out == (OUTV)) {                         \
        hipLaunchKernelGGL((k_march<T, NH, CKV, INITV, RHSV, OUTV>), grid, block, lds, st, a);  \
        return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP;                        \
    }
    // stage operator (top of a cycle)
    FMGMC_MARCH_CASE(true, INIT_LOAD, false, OUT_RESTRICT)
    FMGMC_MARCH_CASE(true, INIT_INTERP, false, OUT_RESTRICT)
    FMGMC_MARCH_CASE(true, INIT_PROLONG, false, OUT_RR | OUT_Q)
    FMGMC_MARCH_CASE(true, INIT_PROLONG, false, 0)
    FMGMC_MARCH_CASE(true, INIT_ZERO, true, OUT_RESTRICT)
    FMGMC_MARCH_CASE(true, INIT_LOAD, true, OUT_RESTRICT)
    FMGMC_MARCH_CASE(true, INIT_PROLONG, true, 0)
    if constexpr (sizeof(T) == 4) {
        // FP32 cycles back to back: prolongation and post-smoothing of one
        // cycle, then pre-smoothing and restriction of the next, in one pass
        FMGMC_MARCH_CASE(true, INIT_PROLONG, true, OUT_RESTRICT)
        if constexpr (NH <= 4) {
            // FP64 refinement of the stage iterate and the pre-smoothing and
            // restriction of the next FP32 cycle, in one pass
            FMGMC_MARCH_CASE(true, INIT_IR, true, OUT_RESTRICT)
            FMGMC_MARCH_CASE(true, INIT_IR, true, OUT_RESTRICT | OUT_PUPD)
            FMGMC_MARCH_CASE(true, INIT_IR, true, OUT_RESTRICT | OUT_FACES)
            FMGMC_MARCH_CASE(true, INIT_IR, true, OUT_RESTRICT | OUT_FACES | OUT_PINTERP)
        }
    }
    if constexpr (sizeof(T) == 8) {
        // the FP64 form's top stage: its first pass also writes the faces on n/2
        FMGMC_MARCH_CASE(true, INIT_INTERP, false, OUT_RESTRICT | OUT_FACES)
    }
    // correction operators (levels below the top)
    FMGMC_MARCH_CASE(false, INIT_ZERO, true, OUT_RESTRICT)
    FMGMC_MARCH_CASE(false, INIT_LOAD, true, OUT_RESTRICT)
    FMGMC_MARCH_CASE(false, INIT_PROLONG, true, 0)
#undef FMGMC_MARCH_CASE
    set_error("launch_march: unsupported variant");
    return FMGMC_EINVAL;
}

template <typename T>
int launch_march(const MarchArgs<T> &a, int S, int nhalf, bool coef_from_k, int init, bool rhs_array,
                 int out, hipStream_t st) {
    if (a.n < 16 || a.n > 1024 || (a.n & (a.n - 1))) {
        set_error("launch_march: n must be a power of two in [16, 1024]");
        return FMGMC_EINVAL;
    }
    if (S <= 0) return FMGMC_OK;
    if (nhalf == 4) return dispatch_march<T, 4>(a, S, coef_from_k, init, rhs_array, out, st);
    if (nhalf == 2) return dispatch_march<T, 2>(a, S, coef_from_k, init, rhs_array, out, st);
    // three and four sweeps: FP32 only (the FP64 register rings would spill)
    if constexpr (std::is_same<T, float>::value) {
        if (nhalf == 6) return dispatch_march<T, 6>(a, S, coef_from_k, init, rhs_array, out, st);
        if (nhalf == 8) return dispatch_march<T, 8>(a, S, coef_from_k, init, rhs_array, out, st);
    }
    set_error("launch_march: nu must be 1 or 2 (FP64) or 1 to 4 (FP32)");
    return FMGMC_EINVAL;
}

template int launch_march<double>(const MarchArgs<double> &, int, int, bool, int, bool, int, hipStream_t);
template int launch_march<float>(const MarchArgs<float> &, int, int, bool, int, bool, int, hipStream_t);

// ------------------------------------------------------------- face pyramid
// Faces of the stage operator on n from K: west face of cell i (i = 0: 2K),
// south face of row j (j = 0: 2K in Case I, no flow in Case II), east and
// north boundary faces 2K (north: 0 in Case II).
template <typename T>
__global__ void k_faces_from_k(int n, const T *__restrict__ K, Faces<T> out, int nc, int all) {
    // coarse cell (I, J) of the n/2 grid from the four faces of the fine operator on it:
    // K of fine rows 2J-1, 2J, 2J+1 at columns 2I-1, 2I, 2I+1 (cell pairs as one load)
    // workgroup -> (sample, chunk of coarse rows), XCD-contiguous: fine row
    // 2J - 1 is also read by the workgroup of coarse row J - 1
    const int u = xcd_unit(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const int s = u / gridDim.x;
    const int c = (u - s * gridDim.x) * blockDim.x + threadIdx.x;
    if (c >= nc * nc) return;
    const int I = c & (nc - 1), J = c >> (31 - __builtin_clz(nc));
    const int i0 = 2 * I, j0 = 2 * J;
    const T *k = K + size_t(s) * n * n;
    const V2<T> r0 = ld2(k + size_t(j0) * n + i0);        // K(i0, j0), K(i0+1, j0)
    const V2<T> r1 = ld2(k + size_t(j0 + 1) * n + i0);    // K(i0, j0+1), K(i0+1, j0+1)
    const V2<T> rs = J > 0 ? ld2(k + size_t(j0 - 1) * n + i0) : r0;  // row j0-1
    const T w0 = I > 0 ? k[size_t(j0) * n + i0 - 1] : r0.a, w1 = I > 0 ? k[size_t(j0 + 1) * n + i0 - 1] : r1.a;
    const T fx0 = I == 0 ? T(2) * r0.a : harm(w0, r0.a);
    const T fx1 = I == 0 ? T(2) * r1.a : harm(w1, r1.a);
    const T fy0 = J == 0 ? (all ? T(2) * r0.a : T(0)) : harm(rs.a, r0.a);
    const T fy1 = J == 0 ? (all ? T(2) * r0.b : T(0)) : harm(rs.b, r0.b);
    const size_t o = size_t(s) * nc * nc + size_t(J) * nc + I;
    out.fx[o] = T(0.5) * (fx0 + fx1);
    out.fy[o] = T(0.5) * (fy0 + fy1);
    if (I == nc - 1) out.fxe[size_t(s) * nc + J] = T(0.5) * (T(2) * r0.b + T(2) * r1.b);
    if (J == nc - 1) out.fyn[size_t(s) * nc + I] = all ? T(0.5) * (T(2) * r1.a + T(2) * r1.b) : T(0);
}

template <typename T>
__global__ void k_faces_coarsen(int n, Faces<T> in, Faces<T> out, int nc) {
    const int u = xcd_unit(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const int s = u / gridDim.x;
    const int c = (u - s * gridDim.x) * blockDim.x + threadIdx.x;
    if (c >= nc * nc) return;
    const int I = c % nc, J = c / nc;
    const size_t fb = size_t(s) * n * n;
    const size_t o = size_t(s) * nc * nc + size_t(J) * nc + I;
    out.fx[o] = T(0.5) * (in.fx[fb + size_t(2 * J) * n + 2 * I] + in.fx[fb + size_t(2 * J + 1) * n + 2 * I]);
    out.fy[o] = T(0.5) * (in.fy[fb + size_t(2 * J) * n + 2 * I] + in.fy[fb + size_t(2 * J) * n + 2 * I + 1]);
    if (I == nc - 1)
        out.fxe[size_t(s) * nc + J] = T(0.5) * (in.fxe[size_t(s) * n + 2 * J] + in.fxe[size_t(s) * n + 2 * J + 1]);
    if (J == nc - 1)
        out.fyn[size_t(s) * nc + I] = T(0.5) * (in.fyn[size_t(s) * n + 2 * I] + in.fyn[size_t(s) * n + 2 * I + 1]);
}

template <typename T>
int launch_faces_from_k(int n, const T *K, int all, Faces<T> out, int S, hipStream_t st) {
    const int nc = n / 2;
    dim3 block(256), grid((nc * nc + 255) / 256, S);
    hipLaunchKernelGGL(k_faces_from_k<T>, grid, block, 0, st, n, K, out, nc, all);
    return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP;
}

template <typename T>
int launch_faces_coarsen(int n, Faces<T> in, Faces<T> out, int S, hipStream_t st) {
    const int nc = n / 2;
    dim3 block(256), grid((nc * nc + 255) / 256, S);
    hipLaunchKernelGGL(k_faces_coarsen<T>, grid, block, 0, st, n, in, out, nc);
    return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP;
}

template int launch_faces_from_k<double>(int, const double *, int, Faces<double>, int, hipStream_t);
template int launch_faces_from_k<float>(int, const float *, int, Faces<float>, int, hipStream_t);
template int launch_faces_coarsen<double>(int, Faces<double>, Faces<double>, int, hipStream_t);
template int launch_faces_coarsen<float>(int, Faces<float>, Faces<float>, int, hipStream_t);

}  // namespace fmgmc
