// Fused red-black Gauss-Seidel passes for the cell-centred five-point
// finite-volume operator (Section 3.1 (1)), used by the V-cycles of the full
// multigrid pass (Section 2.5).
//
// Design (gfx950): one workgroup owns one sample and one lane owns one grid
// column (n <= 1024 lanes). The workgroup marches up the rows. At step F it
// loads row F once from HBM, then applies half-sweep t (t = 1..NH, red first)
// to row F - t. This is the wavefront order of the sweeps, so the result is
// exactly that of NH sequential half-sweeps. The residual follows at row
// F - NH - 1, is summed over 2x2 blocks into the next coarser grid, and/or
// squared into the sample's residual norm.
// Every cell is read and written once per pass: x, K (or the face arrays) and b
// stream through HBM, whatever NH is. Rows in flight live in an LDS ring
// (neighbours in other lanes); per-row coefficients live in a register ring.
// One barrier per row step: every cross-lane read in step F is of data written
// before step F's barrier.
#include "common.h"

namespace fmgmc {

template <typename T>
__device__ __forceinline__ T harm(T a, T b) {
    return T(2) * a * b / (a + b);
}

// coarse value with ghost cells: mirror across north/south, 2 g - v across west/east
template <typename T>
__device__ __forceinline__ T coarse_at(const T *__restrict__ c, int nc, int I, int J, T gW, T gE) {
    J = J < 0 ? 0 : (J >= nc ? nc - 1 : J);
    if (I < 0) return T(2) * gW - c[J * nc];
    if (I >= nc) return T(2) * gE - c[J * nc + nc - 1];
    return c[J * nc + I];
}

// bilinear cell-centred interpolation, weights 9, 3, 3, 1 over 16
template <typename T>
__device__ __forceinline__ T bilinear(const T *__restrict__ c, int nc, int i, int j, T gW, T gE) {
    const int I = i >> 1, J = j >> 1;
    const int di = (i & 1) ? 1 : -1, dj = (j & 1) ? 1 : -1;
    return (T(9) * coarse_at(c, nc, I, J, gW, gE) + T(3) * coarse_at(c, nc, I + di, J, gW, gE) +
            T(3) * coarse_at(c, nc, I, J + dj, gW, gE) + coarse_at(c, nc, I + di, J + dj, gW, gE)) /
           T(16);
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

template <typename T, int NH, bool CK, int INIT, bool RHSA, int OUT>
__global__ __launch_bounds__(1024) void k_march(MarchArgs<T> A) {
    constexpr int R = NH + 3;  // x rows alive in LDS: F - NH - 2 .. F
    constexpr int U = NH + 1;  // coefficient rows alive in registers: F - NH - 1 .. F - 1
    constexpr bool RES = (OUT & (OUT_RESTRICT | OUT_RR)) != 0;
    const int n = A.n;
    const int i = threadIdx.x;
    const int s = blockIdx.x;
    if (A.active && A.active[s] == 0) return;  // uniform over the block

    extern __shared__ unsigned char smem_raw[];
    T *xs = reinterpret_cast<T *>(smem_raw);  // [R][n] x rows
    T *ks = xs + R * n;                       // [3][n] K rows (CK) or west faces
    T *red = ks + 3 * n;                      // [16] reduction scratch

    const size_t base = size_t(s) * n * n;
    const int nc = n >> 1;
    const size_t cbase = size_t(s) * nc * nc;
    const T gW = T(A.pW), gE = T(A.pE);

    // register ring of per-row coefficients, slot = row % U (static after unrolling)
    T tw[U], te[U], tn[U], ts[U], id[U], bv[U];
#pragma unroll
    for (int k = 0; k < U; ++k) { tw[k] = te[k] = tn[k] = ts[k] = id[k] = bv[k] = T(0); }
    T fy_prev = T(0), fy_cur = T(0);  // south faces of rows F-1, F (face mode)
    T b_old = T(0), b_new = T(0);     // rhs of rows F-1, F (array mode)
    T rprev = T(0);                   // residual of the previous (even) row
    T rr = T(0), q = T(0);

    // rhs of a row: given, or the Dirichlet data entering through the side faces
    auto rhs = [&](int slot) -> T {
        if (RHSA) return bv[slot];
        T b0 = T(0);
        if (i == 0) b0 += tw[slot] * gW;
        if (i == n - 1) b0 += te[slot] * gE;
        return b0;
    };
    auto xrow = [&](int row) -> T * { return xs + (row % R) * n; };

    const int LAST = n - 1 + NH + (RES ? 1 : 0);
    for (int F0 = 0; F0 <= LAST; F0 += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int F = F0 + u;
            if (F > LAST) break;
            // ---- 1. load row F
            if (F < n) {
                const size_t idx = base + size_t(F) * n + i;
                T xv;
                if (INIT == INIT_ZERO) xv = T(0);
                else if (INIT == INIT_LOAD) xv = A.x[idx];
                else if (INIT == INIT_PROLONG) xv = A.x[idx] + bilinear(A.xc + cbase, nc, i, F, T(0), T(0));
                else xv = bilinear(A.xc + cbase, nc, i, F, gW, gE);
                xrow(F)[i] = xv;
                if (CK) {
                    ks[(F % 3) * n + i] = A.K[idx];
                } else {
                    ks[(F % 3) * n + i] = A.f.fx[idx];
                    fy_prev = fy_cur;
                    fy_cur = A.f.fy[idx];
                }
                if (RHSA) {
                    b_old = b_new;
                    b_new = A.b[idx];
                }
            } else {
                fy_prev = fy_cur;
                fy_cur = T(0);
                b_old = b_new;
            }
            __syncthreads();
            // ---- 2. coefficients of row r = F - 1
            {
                const int r = F - 1;
                const int sr = (u + U - 1) % U, sp = (u + U - 2) % U;
                if (r >= 0 && r < n) {
                    const T *kr = ks + (r % 3) * n;
                    T w_, e_, n_, s_;
                    if (CK) {
                        const T k0 = kr[i];
                        w_ = (i > 0) ? harm(kr[i - 1], k0) : T(2) * k0;
                        e_ = (i < n - 1) ? harm(k0, kr[i + 1]) : T(2) * k0;
                        n_ = (r + 1 < n) ? harm(k0, ks[((r + 1) % 3) * n + i]) : T(0);
                        s_ = (r > 0) ? tn[sp] : T(0);
                    } else {
                        w_ = kr[i];
                        e_ = (i < n - 1) ? kr[i + 1] : A.f.fxe[size_t(s) * n + r];
                        s_ = fy_prev;
                        n_ = (r + 1 < n) ? fy_cur : T(0);
                    }
                    tw[sr] = w_;
                    te[sr] = e_;
                    tn[sr] = n_;
                    ts[sr] = s_;
                    id[sr] = T(1) / (((w_ + e_) + s_) + n_);
                    if (RHSA) bv[sr] = b_old;
                }
            }
            // ---- 3. half-sweeps: sweep t on row F - t (colour (t-1) & 1)
#pragma unroll
            for (int t = 1; t <= NH; ++t) {
                const int r = F - t;
                if (r >= 0 && r < n && ((i + r) & 1) == ((t - 1) & 1)) {
                    const int sr = (u + 2 * U - t) % U;
                    T *row = xrow(r);
                    T acc = rhs(sr);
                    if (i > 0) acc += tw[sr] * row[i - 1];
                    if (i < n - 1) acc += te[sr] * row[i + 1];
                    if (r > 0) acc += ts[sr] * xrow(r + R - 1)[i];
                    if (r + 1 < n) acc += tn[sr] * xrow(r + 1)[i];
                    row[i] = acc * id[sr];
                }
            }
            // ---- 4. residual of row r = F - NH - 1
            if (RES) {
                const int r = F - NH - 1;
                if (r >= 0 && r < n) {
                    const int sr = (u + 2 * U - NH - 1) % U;
                    const T *row = xrow(r);
                    const T xv = row[i];
                    T acc = rhs(sr);
                    if (i > 0) acc += tw[sr] * row[i - 1];
                    if (i < n - 1) acc += te[sr] * row[i + 1];
                    if (r > 0) acc += ts[sr] * xrow(r + R - 1)[i];
                    if (r + 1 < n) acc += tn[sr] * xrow(r + 1)[i];
                    const T res = acc - (((tw[sr] + te[sr]) + ts[sr]) + tn[sr]) * xv;
                    if (OUT & OUT_RR) rr += res * res;
                    if (OUT & OUT_RESTRICT) {
                        if (r & 1) {
                            T v = res + rprev;
                            v += __shfl_xor(v, 1);
                            if ((i & 1) == 0) A.bc[cbase + size_t(r >> 1) * nc + (i >> 1)] = v;
                        } else {
                            rprev = res;
                        }
                    }
                }
            }
            // ---- 5. write back the finished row F - NH
            {
                const int r = F - NH;
                if (r >= 0 && r < n) {
                    const int sr = (u + 2 * U - NH) % U;
                    const T xv = xrow(r)[i];
                    A.x[base + size_t(r) * n + i] = xv;
                    if ((OUT & OUT_Q) && i == n - 1) q += te[sr] * (xv - gE);
                }
            }
        }
    }
    if (OUT & OUT_RR) {
        const T t = block_sum(rr, red);
        if (threadIdx.x == 0) A.rr[s] = double(t);
    }
    if ((OUT & OUT_Q) && i == n - 1) A.q[s] = double(q);
}

// ------------------------------------------------------------------ dispatch
template <typename T, int NH>
static int dispatch_march(const MarchArgs<T> &a, int S, bool ck, int init, bool rhsa, int out,
                          hipStream_t st) {
    const int n = a.n;
    const size_t lds = (size_t(NH + 3) * n + 3 * n + 16) * sizeof(T);
    dim3 grid(S), block(n);
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
    FMGMC_MARCH_CASE(false, INIT_PROLONG, true, 0)
#undef FMGMC_MARCH_CASE
    set_error("launch_march: unsupported variant");
    return FMGMC_EINVAL;
}

template <typename T>
int launch_march(const MarchArgs<T> &a, int S, int nhalf, bool coef_from_k, int init, bool rhs_array,
                 int out, hipStream_t st) {
    if (a.n < 8 || a.n > 1024 || (a.n & (a.n - 1))) {
        set_error("launch_march: n must be a power of two in [8, 1024]");
        return FMGMC_EINVAL;
    }
    if (S <= 0) return FMGMC_OK;
    if (nhalf == 4) return dispatch_march<T, 4>(a, S, coef_from_k, init, rhs_array, out, st);
    if (nhalf == 2) return dispatch_march<T, 2>(a, S, coef_from_k, init, rhs_array, out, st);
    set_error("launch_march: nu must be 1 or 2");
    return FMGMC_EINVAL;
}

template int launch_march<double>(const MarchArgs<double> &, int, int, bool, int, bool, int, hipStream_t);
template int launch_march<float>(const MarchArgs<float> &, int, int, bool, int, bool, int, hipStream_t);

// ------------------------------------------------------------- face pyramid
// Faces of the stage operator on n from K: west face of cell i (i = 0: 2K),
// south face of row j (j = 0: no flow), east boundary face 2K.
template <typename T>
__global__ void k_faces_from_k(int n, const T *__restrict__ K, Faces<T> out, int nc) {
    // coarse cell (I, J) of the n/2 grid from the four faces of the fine operator on it
    const int s = blockIdx.y;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc * nc) return;
    const int I = c % nc, J = c / nc;
    const T *k = K + size_t(s) * n * n;
    auto kk = [&](int i, int j) { return k[size_t(j) * n + i]; };
    auto fxf = [&](int i, int j) -> T { return i == 0 ? T(2) * kk(0, j) : harm(kk(i - 1, j), kk(i, j)); };
    auto fyf = [&](int i, int j) -> T { return j == 0 ? T(0) : harm(kk(i, j - 1), kk(i, j)); };
    const size_t o = size_t(s) * nc * nc + size_t(J) * nc + I;
    out.fx[o] = T(0.5) * (fxf(2 * I, 2 * J) + fxf(2 * I, 2 * J + 1));
    out.fy[o] = T(0.5) * (fyf(2 * I, 2 * J) + fyf(2 * I + 1, 2 * J));
    if (I == nc - 1)
        out.fxe[size_t(s) * nc + J] = T(0.5) * (T(2) * kk(n - 1, 2 * J) + T(2) * kk(n - 1, 2 * J + 1));
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
}

template <typename T>
int launch_faces_from_k(int n, const T *K, Faces<T> out, int S, hipStream_t st) {
    const int nc = n / 2;
    dim3 block(256), grid((nc * nc + 255) / 256, S);
    hipLaunchKernelGGL(k_faces_from_k<T>, grid, block, 0, st, n, K, out, nc);
    return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP;
}

template <typename T>
int launch_faces_coarsen(int n, Faces<T> in, Faces<T> out, int S, hipStream_t st) {
    const int nc = n / 2;
    dim3 block(256), grid((nc * nc + 255) / 256, S);
    hipLaunchKernelGGL(k_faces_coarsen<T>, grid, block, 0, st, n, in, out, nc);
    return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP;
}

template int launch_faces_from_k<double>(int, const double *, Faces<double>, int, hipStream_t);
template int launch_faces_from_k<float>(int, const float *, Faces<float>, int, hipStream_t);
template int launch_faces_coarsen<double>(int, Faces<double>, Faces<double>, int, hipStream_t);
template int launch_faces_coarsen<float>(int, Faces<float>, Faces<float>, int, hipStream_t);

}  // namespace fmgmc
