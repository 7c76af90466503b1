// Fused red-black Gauss-Seidel passes for the cell-centred five-point
// finite-volume operator (Section 3.1 (1)), used by the V-cycles of the full
// multigrid pass (Section 2.5).
//
// Design (gfx950): one workgroup owns one sample; lane l owns the two cells
// of columns 2l and 2l+1 of every row, one red and one black, so every lane
// updates exactly one cell in every half-sweep. The workgroup marches up the
// rows. At step F it takes row F (loaded NH+1 steps earlier into a register
// queue, so HBM latency overlaps the work of NH+1 rows) and applies half-sweep
// t (t = 1..NH, red first) to row F - t: this is the wavefront order of the
// sweeps, so the result is exactly that of NH sequential half-sweeps. The
// residual follows at row F - NH - 1 and is summed over 2x2 blocks into the
// next coarser grid and/or squared into the sample's residual norm. Every
// cell is read and written once per pass.
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

__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_(double x) {
    // hardware reciprocal refined by two Newton steps (full double precision)
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

template <typename T>
__device__ __forceinline__ T harm(T a, T b) {
    return T(2) * a * b * rcp_(a + b);
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

template <typename T>
__device__ __forceinline__ T block_sum(T v, T *red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
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

template <typename T, int NH, bool CK, int INIT, bool RHSA, int OUT>
__global__ __launch_bounds__(512) void k_march(MarchArgs<T> A) {
    constexpr int U = NH + 1;    // register ring depth = prefetch distance = unroll
    constexpr int RX = march_ring_rows(NH);  // LDS x ring rows (>= NH + 3), power of two
    constexpr bool RES = (OUT & (OUT_RESTRICT | OUT_RR)) != 0;
    constexpr bool CO = (INIT == INIT_PROLONG || INIT == INIT_INTERP);
    constexpr bool LX = (INIT == INIT_LOAD || INIT == INIT_PROLONG);
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
    for (int k = l; k < RX * XS; k += blockDim.x) xs[k] = T(0);
    __syncthreads();

    const size_t base = size_t(s) * n * n;
    const size_t cbase = size_t(s) * nc * nc;
    const T gW = T(A.g.w), gE = T(A.g.e), gS = T(A.g.s), gN = T(A.g.n);
    const bool dns = A.g.all != 0;  // Dirichlet south / north sides (Case I)
    const T cgW = (INIT == INIT_INTERP) ? gW : T(0), cgE = (INIT == INIT_INTERP) ? gE : T(0);
    const T cgS = (INIT == INIT_INTERP) ? gS : T(0), cgN = (INIT == INIT_INTERP) ? gN : T(0);
    const bool first = (l == 0), last = (l == nl - 1);

    // prefetch queue, slot = row % U
    V2<T> qx[U], qk[U], qb[U], qf[U];
    T qc[U], qe[U];
    auto fetch = [&](int slot, int row) {
        const size_t idx = base + size_t(row) * n + 2 * l;
        if (LX) qx[slot] = ld2(A.x + idx);
        if (CK) {
            qk[slot] = ld2(A.K + idx);
        } else {
            qk[slot] = ld2(A.f.fx + idx);
            qf[slot] = ld2(A.f.fy + idx);
            qe[slot] = A.f.fxe[size_t(s) * n + row];
        }
        if (RHSA) qb[slot] = ld2(A.b + idx);
        if (CO) {
            const int J = min((row + 1) >> 1, nc - 1);
            qc[slot] = A.xc[cbase + size_t(J) * nc + l];
        }
    };
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (u < n) fetch(u, u);

    // coefficient ring, slot = row % U: faces west of cell 0, between the cells,
    // east of cell 1; south / north faces and 1/diagonal of both cells; rhs.
    T rw[U], rm[U], re[U], rs0[U], rs1[U], rn0[U], rn1[U], ri0[U], ri1[U], rb0[U], rb1[U];
#pragma unroll
    for (int k = 0; k < U; ++k)
        rw[k] = rm[k] = re[k] = rs0[k] = rs1[k] = rn0[k] = rn1[k] = ri0[k] = ri1[k] = rb0[k] = rb1[k] = T(0);
    V2<T> kprev{T(0), T(0)}, kcur{T(0), T(0)};   // own K (or south faces) of rows F-1, F
    V2<T> bprev{T(0), T(0)}, bcur{T(0), T(0)};
    T eprev = T(0), ecur = T(0);                 // east boundary face of rows F-1, F (correction)
    T rprev = T(0), rr = T(0), q = T(0);

    const int LAST = n - 1 + NH + (RES ? 1 : 0);
    for (int F0 = 0; F0 <= LAST; F0 += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int F = F0 + u;
            if (F > LAST) break;
            T *xrow = xs + (F & (RX - 1)) * XS + 2;
            // ---- 1. take row F from the queue into LDS, refill the slot with row F + U
            kprev = kcur;
            bprev = bcur;
            eprev = ecur;
            V2<T> xraw{T(0), T(0)};
            if (F < n) {
                if (LX) xraw = qx[u];
                if (LX) st2(xrow + 2 * l, xraw.a, xraw.b);
                else if (INIT == INIT_ZERO) st2(xrow + 2 * l, T(0), T(0));
                st2(ks + (F & 3) * n + 2 * l, qk[u].a, qk[u].b);
                kcur = CK ? qk[u] : qf[u];
                if (RHSA) bcur = qb[u];
                if (!CK) ecur = qe[u];
                if (CO) {
                    // coarse row (F+1)/2 into the 4-row ring; the ghost rows -1 and
                    // nc (slots 3 and nc & 3) take the mirror of the edge row
                    // (no flow) or 2 g - it (Dirichlet, Case I)
                    const int Jl = (F + 1) >> 1;
                    const T v = qc[u];
                    cs[(Jl & 3) * nc + l] = (dns && Jl == nc) ? T(2) * cgN - v : v;
                    if (F == 0) cs[3 * nc + l] = dns ? T(2) * cgS - v : v;
                }
                if (F + U < n) fetch(u, F + U);
            } else {
                // past the top row: the north boundary faces (correction operator,
                // Case I) stand in for the next row's south faces, and the ring row
                // above row n-1 is cleared (its slot last held row n - RX, which no
                // step from here on reads)
                kcur = {T(0), T(0)};
                if (F == n) {
                    if (!CK && dns) kcur = ld2(A.f.fyn + size_t(s) * n + 2 * l);
                    st2(xrow + 2 * l, T(0), T(0));
                }
            }
            __syncthreads();
            // ---- 2. coarse-grid correction / FMG interpolation of row F (own cells)
            if (CO && F < n) {
                // J1 = -1 and nc are the ghost rows of the ring; a corner takes the
                // west/east rule applied to the ghost row's edge value
                const int J0 = F >> 1, J1 = J0 + ((F & 1) ? 1 : -1);
                const T *c0 = cs + (J0 & 3) * nc, *c1 = cs + (J1 & 3) * nc;
                const T a0 = c0[l], a1 = c1[l];
                const T w0 = first ? T(2) * cgW - a0 : c0[max(l - 1, 0)];
                const T w1 = first ? T(2) * cgW - a1 : c1[max(l - 1, 0)];
                const T e0 = last ? T(2) * cgE - a0 : c0[min(l + 1, nc - 1)];
                const T e1 = last ? T(2) * cgE - a1 : c1[min(l + 1, nc - 1)];
                const T p0 = (T(9) * a0 + T(3) * w0 + T(3) * a1 + w1) / T(16);
                const T p1 = (T(9) * a0 + T(3) * e0 + T(3) * a1 + e1) / T(16);
                if (INIT == INIT_PROLONG) st2(xrow + 2 * l, xraw.a + p0, xraw.b + p1);
                else st2(xrow + 2 * l, p0, p1);
            }
            // ---- 3. coefficients of row r = F - 1
            {
                const int r = F - 1;
                const int sr = (u + U - 1) % U, sp = (u + U - 2) % U;
                if (r >= 0 && r < n) {
                    const T *kr = ks + (r & 3) * n;
                    T w_, m_, e_, s0, s1, n0, n1;
                    if (CK) {
                        const T k0 = kprev.a, k1 = kprev.b;
                        w_ = first ? T(2) * k0 : harm(kr[max(2 * l - 1, 0)], k0);
                        m_ = harm(k0, k1);
                        e_ = last ? T(2) * k1 : harm(k1, kr[min(2 * l + 2, n - 1)]);
                        n0 = (r + 1 < n) ? harm(k0, kcur.a) : (dns ? T(2) * k0 : T(0));
                        n1 = (r + 1 < n) ? harm(k1, kcur.b) : (dns ? T(2) * k1 : T(0));
                        s0 = (r > 0) ? rn0[sp] : (dns ? T(2) * k0 : T(0));
                        s1 = (r > 0) ? rn1[sp] : (dns ? T(2) * k1 : T(0));
                    } else {
                        w_ = kr[2 * l];
                        m_ = kr[2 * l + 1];
                        e_ = last ? eprev : kr[min(2 * l + 2, n - 1)];
                        s0 = kprev.a;
                        s1 = kprev.b;
                        n0 = kcur.a;
                        n1 = kcur.b;
                    }
                    rw[sr] = w_;
                    rm[sr] = m_;
                    re[sr] = e_;
                    rs0[sr] = s0;
                    rs1[sr] = s1;
                    rn0[sr] = n0;
                    rn1[sr] = n1;
                    ri0[sr] = rcp_(((w_ + m_) + s0) + n0);
                    ri1[sr] = rcp_(((m_ + e_) + s1) + n1);
                    if (RHSA) {
                        rb0[sr] = bprev.a;
                        rb1[sr] = bprev.b;
                    } else {
                        T b0 = first ? w_ * gW : T(0);
                        T b1 = last ? e_ * gE : T(0);
                        if (dns && r == 0) {
                            b0 += s0 * gS;
                            b1 += s1 * gS;
                        }
                        if (dns && r == n - 1) {
                            b0 += n0 * gN;
                            b1 += n1 * gN;
                        }
                        rb0[sr] = b0;
                        rb1[sr] = b1;
                    }
                }
            }
            // ---- 4. half-sweeps: sweep t on row F - t, colour (t-1) & 1
#pragma unroll
            for (int t = 1; t <= NH; ++t) {
                const int r = F - t;
                if (r >= 0 && r < n) {
                    const int sr = (u + 2 * U - t) % U;
                    T *row = xs + (r & (RX - 1)) * XS + 2;
                    const T *up = xs + ((r + 1) & (RX - 1)) * XS + 2;
                    const T *dn = xs + ((r - 1) & (RX - 1)) * XS + 2;
                    // cell pairs are read and written whole: consecutive lanes touch
                    // consecutive 2-cell words, which keeps the LDS accesses
                    // conflict-free; the partner cell is written back unchanged
                    const V2<T> own = ld2(row + 2 * l), vd = ld2(dn + 2 * l), vu = ld2(up + 2 * l);
                    if (((t - 1 + r) & 1) == 0) {  // this lane's red/black cell is column 2l
                        const T west = ld2(row + 2 * l - 2).b;
                        const T v = (((rb0[sr] + rw[sr] * west) + rm[sr] * own.b) + rs0[sr] * vd.a +
                                     rn0[sr] * vu.a) * ri0[sr];
                        st2(row + 2 * l, v, own.b);
                    } else {                        // column 2l + 1
                        const T east = ld2(row + 2 * l + 2).a;
                        const T v = (((rb1[sr] + rm[sr] * own.a) + re[sr] * east) + rs1[sr] * vd.b +
                                     rn1[sr] * vu.b) * ri1[sr];
                        st2(row + 2 * l, own.a, v);
                    }
                }
            }
            // ---- 5. residual of row r = F - NH - 1
            if (RES) {
                const int r = F - NH - 1;
                if (r >= 0 && r < n) {
                    const int sr = (u + 2 * U - NH - 1) % U;
                    const T *row = xs + (r & (RX - 1)) * XS + 2;
                    const T *up = xs + ((r + 1) & (RX - 1)) * XS + 2;
                    const T *dn = xs + ((r - 1) & (RX - 1)) * XS + 2;
                    const V2<T> own = ld2(row + 2 * l), vd = ld2(dn + 2 * l), vu = ld2(up + 2 * l);
                    const T x0 = own.a, x1 = own.b;
                    const T west = ld2(row + 2 * l - 2).b, east = ld2(row + 2 * l + 2).a;
                    const T d0 = ((rw[sr] + rm[sr]) + rs0[sr]) + rn0[sr];
                    const T d1 = ((rm[sr] + re[sr]) + rs1[sr]) + rn1[sr];
                    const T res0 = (((rb0[sr] + rw[sr] * west) + rm[sr] * x1) + rs0[sr] * vd.a + rn0[sr] * vu.a) -
                                   d0 * x0;
                    const T res1 = (((rb1[sr] + rm[sr] * x0) + re[sr] * east) + rs1[sr] * vd.b + rn1[sr] * vu.b) -
                                   d1 * x1;
                    if (OUT & OUT_RR) rr += res0 * res0 + res1 * res1;
                    if (OUT & OUT_RESTRICT) {
                        if (r & 1) A.bc[cbase + size_t(r >> 1) * nc + l] = ((rprev + res0) + res1);
                        else rprev = res0 + res1;
                    }
                }
            }
            // ---- 6. write back the finished row F - NH
            {
                const int r = F - NH;
                if (r >= 0 && r < n) {
                    const int sr = (u + 2 * U - NH) % U;
                    const T *row = xs + (r & (RX - 1)) * XS + 2;
                    const V2<T> xv = ld2(row + 2 * l);
                    const T x0 = xv.a, x1 = xv.b;
                    st2(A.x + base + size_t(r) * n + 2 * l, x0, x1);
                    if (OUT & OUT_Q) {
                        if (!dns) {
                            if (last) q += re[sr] * (x1 - gE);
                        } else if (r == (n >> 1) - 1 || r == (n >> 1)) {
                            // centre cells n/2-1 and n/2: x1 of lane n/4-1, x0 of lane n/4
                            if (l == (n >> 2) - 1) q += x1;
                            else if (l == (n >> 2)) q += x0;
                        }
                    }
                }
            }
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
        (size_t(march_ring_rows(NH)) * (n + 4) + 4 * size_t(n) + 4 * size_t(n / 2) + 16) * sizeof(T);
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
    // coarse cell (I, J) of the n/2 grid from the four faces of the fine operator on it
    const int s = blockIdx.y;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc * nc) return;
    const int I = c % nc, J = c / nc;
    const T *k = K + size_t(s) * n * n;
    auto kk = [&](int i, int j) { return k[size_t(j) * n + i]; };
    auto fxf = [&](int i, int j) -> T { return i == 0 ? T(2) * kk(0, j) : harm(kk(i - 1, j), kk(i, j)); };
    auto fyf = [&](int i, int j) -> T {
        return j == 0 ? (all ? T(2) * kk(i, 0) : T(0)) : harm(kk(i, j - 1), kk(i, j));
    };
    const size_t o = size_t(s) * nc * nc + size_t(J) * nc + I;
    out.fx[o] = T(0.5) * (fxf(2 * I, 2 * J) + fxf(2 * I, 2 * J + 1));
    out.fy[o] = T(0.5) * (fyf(2 * I, 2 * J) + fyf(2 * I + 1, 2 * J));
    if (I == nc - 1)
        out.fxe[size_t(s) * nc + J] = T(0.5) * (T(2) * kk(n - 1, 2 * J) + T(2) * kk(n - 1, 2 * J + 1));
    if (J == nc - 1)
        out.fyn[size_t(s) * nc + I] =
            all ? T(0.5) * (T(2) * kk(2 * I, n - 1) + T(2) * kk(2 * I + 1, n - 1)) : T(0);
}

template <typename T>
__global__ void k_faces_coarsen(int n, Faces<T> in, Faces<T> out, int nc) {
    const int s = blockIdx.y;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
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
