// Small grids (n <= 32): one workgroup holds a sample's whole sub-hierarchy
// in LDS and runs a complete cycle (V(nu1,nu2), with W-cycle coarse-grid
// corrections on grids n <= wmax): red-black Gauss-Seidel,
// residual restriction by 2x2 sums, bilinear prolongation, and the direct
// solve on the coarsest grid (Section 2.5; Cholesky factor precomputed in
// FP64, applied as the explicit inverse of the 16 x 16 coarsest operator,
// built once per batch from its Cholesky factor). With top == 0 the call is the
// coarsest-grid direct solve itself (the first stage of full multigrid).
// One 256-lane workgroup per sample. Boundary conditions of Case II or Case I
// (Table 1): a boundary face enters the diagonal and the right-hand side.
#include "common.h"

namespace fmgmc {

namespace {

constexpr int kMaxLev = 4;   // 4, 8, 16, 32
constexpr int kThreads = 256;
// FP64: the top grid's right-hand side is not kept in LDS (a lane reads only
// its own cells' values): the kSw cells of each colour that a lane updates in
// a half-sweep hold theirs in registers (n <= 32: n^2 / 2 <= kSw kThreads);
// the restriction and the residual norm, once per call, read or form it again.
// A 32^2 sample then takes 36 KB of LDS instead of 44 KB, four per CU instead
// of three (k_small<double> 210 -> 186 us per 4096-sample call, bitwise
// unchanged). In FP32 the same registers took the kernel from 62 to 77 VGPRs,
// six waves per SIMD instead of eight, and it ran slower (118 -> 135 us; capped
// at 64 VGPRs it spilled, 146 us), so FP32 keeps it in LDS (seven samples per CU).
constexpr int kSw = 2;

template <typename T>
__device__ __forceinline__ T harm_s(T a, T b) {
    return T(2) * a * b / (a + b);
}

template <typename T>
struct Lv {
    int n, lg;  // n = 2^lg cells per side
    T *x, *b, *fx, *fy, *fxe, *fyn;
};

// boundary values used by an interpolation (0 for a correction)
template <typename T>
struct G4 {
    T w, e, s, n;
    bool all;
};

// value in coarse row J (a ghost row beyond the south / north side: a mirror
// for no flow, 2 g - value for Dirichlet), then beyond the west / east side
// 2 g - that row's edge value
template <typename T>
__device__ __forceinline__ T ghost_row(const T *c, int nc, int I, int J, const G4<T> &g) {
    if (J >= 0 && J < nc) return c[J * nc + I];
    const int Jc = J < 0 ? 0 : nc - 1;
    return g.all ? T(2) * (J < 0 ? g.s : g.n) - c[Jc * nc + I] : c[Jc * nc + I];
}

template <typename T>
__device__ __forceinline__ T ghost_at(const T *c, int nc, int I, int J, const G4<T> &g) {
    if (I < 0) return T(2) * g.w - ghost_row(c, nc, 0, J, g);
    if (I >= nc) return T(2) * g.e - ghost_row(c, nc, nc - 1, J, g);
    return ghost_row(c, nc, I, J, g);
}

template <typename T>
__device__ __forceinline__ T interp_at(const T *c, int nc, int i, int j, const G4<T> &g) {
    const int I = i >> 1, J = j >> 1;
    const int di = (i & 1) ? 1 : -1, dj = (j & 1) ? 1 : -1;
    return (T(9) * ghost_at(c, nc, I, J, g) + T(3) * ghost_at(c, nc, I + di, J, g) +
            T(3) * ghost_at(c, nc, I, J + dj, g) + ghost_at(c, nc, I + di, J + dj, g)) /
           T(16);
}

// bilinear prolongation of a correction (homogeneous boundary data): the
// ghost value beyond a Dirichlet side is minus the edge value, beyond a
// no-flow side the edge value itself (interp_at with zero data, without its
// branches)
template <typename T>
__device__ __forceinline__ T prolong_at(const T *c, int nc, int lgc, int i, int j, bool all) {
    const int I = i >> 1, J = j >> 1;
    const int I1 = I + ((i & 1) ? 1 : -1), J1 = J + ((j & 1) ? 1 : -1);
    const bool ox = I1 < 0 || I1 >= nc, oy = J1 < 0 || J1 >= nc;
    const int Ic = ox ? I : I1, Jc = oy ? J : J1;
    const T a = c[(J << lgc) + I];
    T bx = c[(J << lgc) + Ic], by = c[(Jc << lgc) + I], bxy = c[(Jc << lgc) + Ic];
    if (ox) {
        bx = -bx;
        bxy = -bxy;
    }
    if (oy && all) {
        by = -by;
        bxy = -bxy;
    }
    return (T(9) * a + T(3) * bx + T(3) * by + bxy) / T(16);
}

// sum over interior neighbours of T_nb x_nb, plus the right-hand side bv of
// the cell (a side without an interior neighbour adds 0 * x of the cell
// itself, so every lane runs the same instructions and the sum keeps its order)
template <typename T>
__device__ __forceinline__ T nbsum(const Lv<T> &L, int i, int j, T bv) {
    const int n = L.n, P = j * n + i;
    const bool w = i > 0, e = i < n - 1, so = j > 0, no = j < n - 1;
    const T tw = w ? L.fx[P] : T(0), te = e ? L.fx[P + 1] : T(0);
    const T ts = so ? L.fy[P] : T(0), tn = no ? L.fy[P + n] : T(0);
    T acc = bv;
    acc += tw * L.x[w ? P - 1 : P];
    acc += te * L.x[e ? P + 1 : P];
    acc += ts * L.x[so ? P - n : P];
    acc += tn * L.x[no ? P + n : P];
    return acc;
}

template <typename T>
__device__ __forceinline__ T diag(const Lv<T> &L, int i, int j) {
    const int n = L.n, P = j * n + i;
    const T te = (i < n - 1) ? L.fx[P + 1] : L.fxe[j];
    const T tn = (j < n - 1) ? L.fy[P + n] : L.fyn[i];
    return ((L.fx[P] + te) + L.fy[P]) + tn;
}

// right-hand side from bt[m] (breg: the top grid's, in registers) or L.b
template <typename T, int COLOUR>
__device__ __forceinline__ void half_sweep(const Lv<T> &L, int tid, const T (&bt)[kSw], bool breg) {
    const int n = L.n, h = n >> 1;
    if constexpr (sizeof(T) == 8) {
#pragma unroll
        for (int m = 0; m < kSw; ++m) {
            const int c = tid + m * kThreads;
            if (c < n * h) {
                const int j = c >> (L.lg - 1), i = 2 * (c & (h - 1)) + ((j + COLOUR) & 1);
                L.x[j * n + i] = nbsum(L, i, j, breg ? bt[m] : L.b[j * n + i]) * rcp_(diag(L, i, j));
            }
        }
    } else {
        for (int c = tid; c < n * h; c += kThreads) {
            const int j = c >> (L.lg - 1), i = 2 * (c & (h - 1)) + ((j + COLOUR) & 1);
            L.x[j * n + i] = nbsum(L, i, j, L.b[j * n + i]) * rcp_(diag(L, i, j));
        }
    }
    __syncthreads();
}

template <typename T>
__device__ void smooth(const Lv<T> &L, int nu, int tid, const T (&bt)[2][kSw], bool breg) {
    for (int k = 0; k < nu; ++k) {
        half_sweep<T, 0>(L, tid, bt[0], breg);
        half_sweep<T, 1>(L, tid, bt[1], breg);
    }
}

// coarsest solve x = A^{-1} b in FP64 on the 4 x 4 grid: one lane per
// unknown (A^{-1} read from global memory, where it stays in cache: it is
// 2 KB per sample). The row is loaded whole before the products, so its loads
// overlap; the sum runs in k order.
constexpr int kN0 = 16;  // unknowns of the coarsest grid
template <typename T>
__device__ void coarse_solve(const double *Ainv, const T *b, T *x, int tid) {
    if (tid < kN0) {
        const double *row = Ainv + tid * kN0;
        double a[kN0];
        T bv[kN0];
#pragma unroll
        for (int k = 0; k < kN0; ++k) a[k] = row[k];
#pragma unroll
        for (int k = 0; k < kN0; ++k) bv[k] = b[k];
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < kN0; ++k) s += a[k] * double(bv[k]);
        x[tid] = T(s);
    }
    __syncthreads();
}

template <typename T>
__host__ __device__ constexpr bool small_rhs_in_registers(int top) { return sizeof(T) == 8 && top > 0; }

template <typename T>
__global__ __launch_bounds__(kThreads) void k_small(SmallArgs<T> A, int init, bool rhs_array, int out) {
    const int s = blockIdx.x;
    if (A.active && A.active[s] == 0) return;
    const int tid = threadIdx.x;
    extern __shared__ unsigned char smem_raw[];
    T *const base = reinterpret_cast<T *>(smem_raw);
    const int top = A.top;
    // FP64: the top grid's right-hand side in registers (above the coarsest grid,
    // whose direct solve reads all of it in every lane)
    const bool breg = small_rhs_in_registers<T>(top);
    // level k arrays (x, b, fx, fy of n*n, then fxe and fyn of n; no b on the top
    // grid with breg), packed from level 0 up; 1/diagonal is recomputed where
    // needed: both keep more samples resident per CU
    auto lv = [&](int k) -> Lv<T> {
        T *p = base;
        for (int j = 0; j < k; ++j) p += 4 * A.ns[j] * A.ns[j] + 2 * A.ns[j];
        const int n = A.ns[k];
        Lv<T> L;
        L.n = n;
        L.lg = __builtin_ctz(n);
        L.x = p; p += n * n;
        if (k == top && breg) {
            L.b = nullptr;
        } else {
            L.b = p;
            p += n * n;
        }
        L.fx = p; p += n * n;
        L.fy = p; p += n * n;
        L.fxe = p; p += n;
        L.fyn = p;
        return L;
    };
    T *p = base;
    for (int j = 0; j <= top; ++j) p += ((j == top && breg) ? 3 : 4) * A.ns[j] * A.ns[j] + 2 * A.ns[j];
    T *red = p;
    const int N0 = A.ns[0] * A.ns[0];
    const double *Ls = A.chol + size_t(s) * N0 * N0;
    const bool dns = A.g.all != 0;
    const G4<T> gsol{T(A.g.w), T(A.g.e), T(A.g.s), T(A.g.n), dns};
    const G4<T> gzero{T(0), T(0), T(0), T(0), dns};
    // coefficients of every level
    for (int k = 0; k <= top; ++k) {
        const Lv<T> Lk = lv(k);
        const int n = Lk.n, nn = n * n;
        if (k == top && A.top_from_k) {
            const T *K = A.Ktop + size_t(s) * nn;
#pragma unroll 4
            for (int c = tid; c < nn; c += kThreads) {
                const int i = c & (n - 1), j = c >> Lk.lg;
                // the west and south neighbours' K, loaded without a branch (own K at an edge)
                const T kc = K[c], kw = K[i > 0 ? c - 1 : c], ksn = K[j > 0 ? c - n : c];
                Lk.fx[c] = i == 0 ? T(2) * kc : harm_s(kw, kc);
                Lk.fy[c] = j == 0 ? (dns ? T(2) * kc : T(0)) : harm_s(ksn, kc);
                if (i == n - 1) Lk.fxe[j] = T(2) * kc;
                if (j == n - 1) Lk.fyn[i] = dns ? T(2) * kc : T(0);
            }
        } else {
            const T *fx = A.f[k].fx + size_t(s) * nn, *fy = A.f[k].fy + size_t(s) * nn;
            const T *fe = A.f[k].fxe + size_t(s) * n, *fn = A.f[k].fyn + size_t(s) * n;
#pragma unroll 4
            for (int c = tid; c < nn; c += kThreads) {
                Lk.fx[c] = fx[c];
                Lk.fy[c] = fy[c];
            }
            for (int c = tid; c < n; c += kThreads) {
                Lk.fxe[c] = fe[c];
                Lk.fyn[c] = fn[c];
            }
        }
    }
    __syncthreads();
    // right-hand side of the top grid at cell (i, j): the array, or the boundary
    // data through the boundary faces
    const Lv<T> Tp = lv(top);
    auto top_rhs = [&](int i, int j) -> T {
        const int n = Tp.n, c = j * n + i;
        if (rhs_array) return A.b[size_t(s) * n * n + c];
        T b0 = T(0);
        if (i == 0) b0 += Tp.fx[c] * gsol.w;
        if (i == n - 1) b0 += Tp.fxe[j] * gsol.e;
        if (dns && j == 0) b0 += Tp.fy[c] * gsol.s;
        if (dns && j == n - 1) b0 += Tp.fyn[i] * gsol.n;
        return b0;
    };
    // right-hand side (in LDS, or the half-sweeps' cells in registers) and
    // initial guess on the top level
    T bsw[2][kSw];
    {
        const int n = Tp.n, nn = n * n, h = n >> 1;
        if (breg) {
#pragma unroll
            for (int col = 0; col < 2; ++col)
#pragma unroll
                for (int m = 0; m < kSw; ++m) {
                    const int c = tid + m * kThreads;
                    const int j = c >> (Tp.lg - 1), i = 2 * (c & (h - 1)) + ((j + col) & 1);
                    bsw[col][m] = c < n * h ? top_rhs(i, j) : T(0);
                }
        }
#pragma unroll 4
        for (int c = tid; c < nn; c += kThreads) {
            const int i = c & (n - 1), j = c >> Tp.lg;
            if (!breg) Tp.b[c] = top_rhs(i, j);
            T xv = T(0);
            if (init == INIT_LOAD) xv = A.x[size_t(s) * nn + c];
            else if (init == INIT_INTERP) xv = interp_at(A.xc + size_t(s) * (nn / 4), n / 2, i, j, gsol);
            Tp.x[c] = xv;
        }
    }
    __syncthreads();

    // Cycle on levels top..0, iterative: descending from level k runs the
    // pre-smoothing and restriction, then cnt[k] coarse cycles (two when the
    // coarse grid is not the coarsest and has n <= wmax, a W-cycle; else one),
    // then prolongation and post-smoothing. Control flow is uniform.
    unsigned cnt = 0;  // 2 bits per level: coarse cycles still to run from that level
    int k = top;
    bool down = true;
    while (true) {
        if (down) {
            if (k == 0) {
                const Lv<T> L0 = lv(0);
                coarse_solve(Ls, L0.b, L0.x, tid);
                if (top == 0) break;
                k = 1;
                down = false;
                continue;
            }
            const Lv<T> Lk = lv(k), Lc = lv(k - 1);
            const bool kb = breg && k == top;
            smooth(Lk, A.nu1, tid, bsw, kb);
            const int n = Lk.n, nc = n / 2;
            for (int c = tid; c < nc * nc; c += kThreads) {  // one coarse cell per lane
                const int I = c & (nc - 1), J = c >> (Lk.lg - 1);
                T acc = T(0);
                for (int dj = 0; dj < 2; ++dj)
                    for (int di = 0; di < 2; ++di) {
                        const int i = 2 * I + di, j = 2 * J + dj;
                        const T bv = kb ? top_rhs(i, j) : Lk.b[j * n + i];
                        acc += nbsum(Lk, i, j, bv) - diag(Lk, i, j) * Lk.x[j * n + i];
                    }
                Lc.b[c] = acc;
                Lc.x[c] = T(0);
            }
            __syncthreads();
            const unsigned g = (k - 1 > 0 && Lc.n <= A.wmax) ? 2u : 1u;
            cnt = (cnt & ~(3u << (2 * k))) | (g << (2 * k));
            k = k - 1;
        } else {
            const unsigned left = ((cnt >> (2 * k)) & 3u) - 1u;
            cnt = (cnt & ~(3u << (2 * k))) | (left << (2 * k));
            if (left > 0) {  // run the coarse cycle again from its current iterate
                k = k - 1;
                down = true;
                continue;
            }
            const Lv<T> Lk = lv(k), Lc = lv(k - 1);
            const int n = Lk.n, nc = n / 2;
            for (int c = tid; c < n * n; c += kThreads)
                Lk.x[c] += prolong_at(Lc.x, nc, Lc.lg, c & (n - 1), c >> Lk.lg, dns);
            __syncthreads();
            smooth(Lk, A.nu2, tid, bsw, breg && k == top);
            if (k == top) break;
            k = k + 1;
        }
    }

    // outputs
    const int n = Tp.n, nn = n * n;
    for (int c = threadIdx.x; c < nn; c += kThreads) A.x[size_t(s) * nn + c] = Tp.x[c];
    if (out & OUT_RR) {
        T rr = T(0);
        for (int c = threadIdx.x; c < nn; c += kThreads) {
            const int i = c & (n - 1), j = c >> Tp.lg;
            const T r = nbsum(Tp, i, j, breg ? top_rhs(i, j) : Tp.b[c]) - diag(Tp, i, j) * Tp.x[c];
            rr += r * r;
        }
        for (int o = 32; o > 0; o >>= 1) rr += __shfl_xor(rr, o);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rr;
        __syncthreads();
        if (threadIdx.x == 0) {
            T t = T(0);
            for (int w = 0; w < kThreads / 64; ++w) t += red[w];
            A.rr[s] = double(t);
        }
    }
    if ((out & OUT_Q) && threadIdx.x == 0) {
        T q = T(0);
        if (dns) {
            const int m = n >> 1;  // centre cells m-1, m (n >= 4)
            q = ((Tp.x[(m - 1) * n + m - 1] + Tp.x[m * n + m - 1]) + (Tp.x[(m - 1) * n + m] + Tp.x[m * n + m])) *
                T(0.25);
        } else {
            for (int j = 0; j < n; ++j) q += Tp.fxe[j] * (Tp.x[j * n + n - 1] - gsol.e);
        }
        A.q[s] = double(q);
    }
}

}  // namespace

template <typename T>
int launch_small(const SmallArgs<T> &a, int S, int init, bool rhs_array, int out, hipStream_t st) {
    if (a.top < 0 || a.top >= kMaxLev || a.ns[0] * a.ns[0] != kN0) {
        set_error("launch_small: unsupported hierarchy");
        return FMGMC_EINVAL;
    }
    if (S <= 0) return FMGMC_OK;
    size_t words = 0;
    for (int k = 0; k <= a.top; ++k)
        words += ((k == a.top && small_rhs_in_registers<T>(a.top)) ? 3 : 4) * size_t(a.ns[k]) * a.ns[k] +
                 2 * size_t(a.ns[k]);
    const size_t bytes = (words + 8) * sizeof(T);  // the levels, then 8 reduction slots
    hipLaunchKernelGGL(k_small<T>, dim3(S), dim3(kThreads), bytes, st, a, init, rhs_array, out);
    return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP;
}

template int launch_small<double>(const SmallArgs<double> &, int, int, bool, int, hipStream_t);
template int launch_small<float>(const SmallArgs<float> &, int, int, bool, int, hipStream_t);

// ------------------------------------------------- coarsest operator inverse
// One wave per sample, the N x N (N = n0^2 <= 16) operator in LDS: assembly
// (one lane per cell), lower Cholesky column by column (lanes over the rows
// below the diagonal), the columns of L^{-1} by forward substitution (one
// lane per column), then A^{-1} = L^{-T} L^{-1} (lanes over the entries).
template <typename T>
__global__ __launch_bounds__(64) void k_chol(int n0, const T *K, Faces<T> f, bool from_k, int all, double *Lout) {
    __shared__ double L[16 * 16];
    __shared__ double Li[16 * 16];
    const int s = blockIdx.x, t = threadIdx.x;
    const int N = n0 * n0;
    auto fxv = [&](int i, int j) -> double {
        if (from_k) {
            const T *k = K + size_t(s) * N;
            return i == 0 ? 2.0 * double(k[j * n0]) : double(harm_s(k[j * n0 + i - 1], k[j * n0 + i]));
        }
        return double(f.fx[size_t(s) * N + j * n0 + i]);
    };
    auto fxe = [&](int j) -> double {
        if (from_k) return 2.0 * double(K[size_t(s) * N + j * n0 + n0 - 1]);
        return double(f.fxe[size_t(s) * n0 + j]);
    };
    auto fyv = [&](int i, int j) -> double {  // south face of cell (i, j), j = n0: north boundary
        if (from_k) {
            const T *k = K + size_t(s) * N;
            if (j == 0) return all ? 2.0 * double(k[i]) : 0.0;
            if (j == n0) return all ? 2.0 * double(k[(n0 - 1) * n0 + i]) : 0.0;
            return double(harm_s(k[(j - 1) * n0 + i], k[j * n0 + i]));
        }
        if (j == n0) return double(f.fyn[size_t(s) * n0 + i]);
        return double(f.fy[size_t(s) * N + j * n0 + i]);
    };
    for (int e = t; e < N * N; e += 64) L[e] = 0.0;
    __syncthreads();
    if (t < N) {
        const int P = t, i = P % n0, j = P / n0;
        const double w = fxv(i, j), e = (i < n0 - 1) ? fxv(i + 1, j) : fxe(j);
        const double so = fyv(i, j), no = fyv(i, j + 1);
        L[P * N + P] = ((w + e) + so) + no;
        if (i > 0) L[P * N + P - 1] = -w;
        if (j > 0) L[P * N + P - n0] = -so;
    }
    __syncthreads();
    for (int c = 0; c < N; ++c) {
        if (t == 0) {
            double d = L[c * N + c];
            for (int k = 0; k < c; ++k) d -= L[c * N + k] * L[c * N + k];
            L[c * N + c] = sqrt(d);  // NaN for a non-SPD (non-finite) operator; flagged by the residual check
        }
        __syncthreads();
        if (t > c && t < N) {
            double v = L[t * N + c];
            for (int k = 0; k < c; ++k) v -= L[t * N + k] * L[c * N + k];
            L[t * N + c] = v / L[c * N + c];
        }
        __syncthreads();
    }
    if (t < N) {
        const int c = t;  // column c of L^{-1}, kept in Li[.][c]
        for (int r = 0; r < N; ++r) {
            double v = (r == c) ? 1.0 : 0.0;
            for (int k = c; k < r; ++k) v -= L[r * N + k] * Li[k * N + c];
            Li[r * N + c] = (r < c) ? 0.0 : v / L[r * N + r];
        }
    }
    __syncthreads();
    double *out = Lout + size_t(s) * N * N;
    for (int e = t; e < N * N; e += 64) {
        const int i = e / N, j = e % N;
        double v = 0.0;
        for (int k = (i > j ? i : j); k < N; ++k) v += Li[k * N + i] * Li[k * N + j];
        out[e] = v;
    }
}

template <typename T>
int launch_chol(int n0, const T *K, Faces<T> f, bool from_k, int all, double *L, int S, hipStream_t st) {
    if (n0 * n0 > 16) {
        set_error("launch_chol: coarsest grid too large");
        return FMGMC_EINVAL;
    }
    if (S <= 0) return FMGMC_OK;
    hipLaunchKernelGGL(k_chol<T>, dim3(S), dim3(64), 0, st, n0, K, f, from_k, all, L);
    return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP;
}

template int launch_chol<double>(int, const double *, Faces<double>, bool, int, double *, int, hipStream_t);
template int launch_chol<float>(int, const float *, Faces<float>, bool, int, double *, int, hipStream_t);

}  // namespace fmgmc
