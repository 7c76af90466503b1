// FP64 iterative refinement around FP32 V-cycles, FMG interpolation into
// FP64, right-hand-side norms, per-sample convergence bookkeeping and the
// compensated estimator reductions (Section 2.1 Eqs. (3)-(5), Section 2.4).
#include <cmath>
#include <mutex>
#include <type_traits>

#include "common.h"

namespace fmgmc {

namespace {

// transmissibility 2ab/(a+b) through the refined reciprocal, as in the
// marching passes (so the fused refinement forms the same operator)
__device__ __forceinline__ double harm_d(double a, double b) { return 2.0 * a * b * rcp_(a + b); }

// Refinement pass, marching over rows (one workgroup per sample, one lane per
// column): p <- p + e; r = b - A p in FP64 with the stage operator; r is
// handed to the next FP32 cycles, ||r||^2 and the QoI accumulate (east
// outflow in Case II, the centre pressure in Case I).
__global__ __launch_bounds__(1024) void k_ir(IRArgs A) {
    const int n = A.n, i = threadIdx.x, s = blockIdx.x;
    if (A.active && A.active[s] == 0) return;
    extern __shared__ unsigned char smem_raw[];
    double *ps = reinterpret_cast<double *>(smem_raw);  // [3][n]
    double *ks = ps + 3 * n;                            // [3][n]
    double *red = ks + 3 * n;                           // [18]: 16 wave partials, 2 QoI partials
    const bool dns = A.g.all != 0;
    const size_t base = size_t(s) * n * n;
    double rr = 0.0, q = 0.0;
    double tn_prev = 0.0;
    // rows F + 1 .. F + D are in flight in a register queue (slot = row % D)
    constexpr int D = 4;
    double qp[D], qk[D];
    float qe[D];
    auto fetch = [&](int slot, int row) {
        const size_t idx = base + size_t(row) * n + i;
        qp[slot] = __builtin_nontemporal_load(A.p + idx);
        if (A.e) qe[slot] = __builtin_nontemporal_load(A.e + idx);
        qk[slot] = __builtin_nontemporal_load(A.K + idx);
    };
#pragma unroll
    for (int d = 0; d < D; ++d)
        if (d < n) fetch(d, d);
    // step F: row F enters the LDS ring, the residual of row F - 1 is formed. With
    // C (checked) the row indices are range-tested; without, valid for 2 <= F and
    // F + D < n, the step is straight-line code and no prefetch is conditional.
    auto step = [&](const int F, const int u, auto chk) {
        constexpr bool C = decltype(chk)::value;
        if (!C || F < n) {
            double pv = qp[u];
            if (A.e) pv += double(qe[u]);
            ps[(F % 3) * n + i] = pv;
            ks[(F % 3) * n + i] = qk[u];
            if (!C || F + D < n) fetch(u, F + D);
        }
        __syncthreads();
        const int r = F - 1;
        if (!C || r >= 0) {
            const double *kr = ks + (r % 3) * n, *pr = ps + (r % 3) * n;
            const double k0 = kr[i], x0 = pr[i];
            const double tw = (i > 0) ? harm_d(kr[i - 1], k0) : 2.0 * k0;
            const double te = (i < n - 1) ? harm_d(k0, kr[i + 1]) : 2.0 * k0;
            const double tn = (!C || r + 1 < n) ? harm_d(k0, ks[(F % 3) * n + i]) : (dns ? 2.0 * k0 : 0.0);
            const double ts = (!C || r > 0) ? tn_prev : (dns ? 2.0 * k0 : 0.0);
            double acc = 0.0;
            if (i == 0) acc += tw * A.g.w;
            if (i == n - 1) acc += te * A.g.e;
            if (C && dns && r == 0) acc += ts * A.g.s;
            if (C && dns && r == n - 1) acc += tn * A.g.n;
            if (i > 0) acc += tw * pr[i - 1];
            if (i < n - 1) acc += te * pr[i + 1];
            if (!C || r > 0) acc += ts * ps[((r + 2) % 3) * n + i];
            if (!C || r + 1 < n) acc += tn * ps[(F % 3) * n + i];
            const double res = acc - (((tw + te) + ts) + tn) * x0;
            rr += res * res;
            // streamed results (read back only by a later pass): non-temporal stores
            __builtin_nontemporal_store(float(res), A.r32 + base + size_t(r) * n + i);
            if (A.e) __builtin_nontemporal_store(x0, A.p + base + size_t(r) * n + i);
            if (!dns) {
                if (i == n - 1) q += te * (x0 - A.g.e);
            } else if ((r == (n >> 1) - 1 || r == (n >> 1)) && (i == (n >> 1) - 1 || i == (n >> 1))) {
                q += x0;
            }
            tn_prev = tn;
        }
    };
    const int lo = D;                          // first unchecked step (D >= 2)
    const int hi = max(lo, ((n - D) / D) * D); // first checked step after them
    int F0 = 0;
    for (; F0 < lo; F0 += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) step(F0 + u, u, std::true_type{});
    }
    for (; F0 < hi; F0 += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) step(F0 + u, u, std::false_type{});
    }
    for (; F0 <= n; F0 += D) {
#pragma unroll
        for (int u = 0; u < D; ++u)
            if (F0 + u <= n) step(F0 + u, u, std::true_type{});
    }
    // butterfly over the wave's lanes of this workgroup (n lanes when n < 64)
    for (int o = min(32, n >> 1); o > 0; o >>= 1) rr += __shfl_xor(rr, o);
    __syncthreads();
    if ((i & 63) == 0) red[i >> 6] = rr;
    __syncthreads();
    if (i == 0) {
        double t = 0.0;
        for (int w = 0; w < (n + 63) / 64; ++w) t += red[w];
        A.rr[s] = t;
    }
    if (!dns) {
        if (i == n - 1) A.q[s] = q;
    } else {
        // centre columns n/2 - 1 and n/2, each summed over the two centre rows
        if (i == (n >> 1) - 1) red[16] = q;
        if (i == (n >> 1)) red[17] = q;
        __syncthreads();
        if (i == 0) A.q[s] = (red[16] + red[17]) * 0.25;
    }
}

// One thread per coarse cell (I, J): its 2 x 2 fine cells from the 3 x 3
// coarse neighbourhood (ghost values at the boundary), written as two
// 16-byte row pairs.
template <typename TS>
__global__ void k_interp64(int n, const TS *xc, double *p, const int32_t *active, Bnd g) {
    // workgroup -> (sample, chunk of coarse rows), XCD-contiguous: the three
    // workgroups that read a coarse row share an L2
    const int u = xcd_unit(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const int s = u / gridDim.x, bx = u - s * gridDim.x;
    if (active && active[s] == 0) return;
    const int nc = n / 2;
    const int c = bx * blockDim.x + threadIdx.x;
    if (c >= nc * nc) return;
    const int lgc = 31 - __builtin_clz(nc);
    const int I = c & (nc - 1), J = c >> lgc;
    const TS *x = xc + size_t(s) * nc * nc;
    // the 3 x 3 coarse neighbourhood with ghosts: beyond the south / north
    // side a mirror (no flow) or 2 g - value (Dirichlet), then beyond the
    // west / east side 2 g - the edge value of that (possibly ghost) row;
    // taken from the clamped neighbour by selects, so every lane runs the
    // same instructions
    double v[3][3];
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj) {
        const int Jn = J + dj;
        const bool oy = Jn < 0 || Jn >= nc;
        const int Jc = oy ? J : Jn;
        const bool fy = oy && g.all;
        const double ay = fy ? 2.0 * (Jn < 0 ? g.s : g.n) : 0.0;
#pragma unroll
        for (int di = -1; di <= 1; ++di) {
            const int In = I + di;
            const bool ox = In < 0 || In >= nc;
            const int Ic = ox ? I : In;
            const double cv = double(x[(Jc << lgc) + Ic]);
            const double row = fy ? ay - cv : cv;
            v[dj + 1][di + 1] = ox ? 2.0 * (In < 0 ? g.w : g.e) - row : row;
        }
    }
    double *o = p + size_t(s) * n * n + size_t(2 * J) * n + 2 * I;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int dj = b ? 1 : -1;
        double out[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int di = a ? 1 : -1;
            out[a] = (9.0 * v[1][1] + 3.0 * v[1][1 + di] + 3.0 * v[1 + dj][1] + v[1 + dj][1 + di]) / 16.0;
        }
        typedef double d2v __attribute__((ext_vector_type(2)));
        __builtin_nontemporal_store(d2v{out[0], out[1]}, reinterpret_cast<d2v *>(o + size_t(b) * n));
    }
}

// one workgroup per sample, lanes over the rows (column 0 and n-1 of each row);
// in Case I also over the columns of rows 0 and n-1, the corner cells taking
// both of their boundary faces
template <typename T>
__global__ __launch_bounds__(256) void k_bnorm(int n, const T *K, Bnd g, double *bn) {
    __shared__ double red[4];
    const int s = blockIdx.x;
    const T *k = K + size_t(s) * n * n;
    auto kv = [&](int i, int j) { return 2.0 * double(k[size_t(j) * n + i]); };
    double acc = 0.0;
    if (!g.all) {
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            const double bw = kv(0, j) * g.w;
            const double be = kv(n - 1, j) * g.e;
            acc += bw * bw + be * be;
        }
    } else {
        for (int t = threadIdx.x; t < 4 * n; t += blockDim.x) {
            // t < 2n: cell (i, 0) or (i, n-1); else the west / east cell of rows 1..n-2
            int i, j;
            if (t < 2 * n) {
                i = t % n;
                j = (t < n) ? 0 : n - 1;
            } else {
                const int u = t - 2 * n;
                j = 1 + (u >> 1);
                if (j > n - 2) continue;
                i = (u & 1) ? n - 1 : 0;
            }
            double b = 0.0;
            if (i == 0) b += kv(i, j) * g.w;
            if (i == n - 1) b += kv(i, j) * g.e;
            if (j == 0) b += kv(i, j) * g.s;
            if (j == n - 1) b += kv(i, j) * g.n;
            acc += b * b;
        }
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) bn[s] = sqrt(((red[0] + red[1]) + red[2]) + red[3]);
}

__global__ __launch_bounds__(1024) void k_check(CheckArgs A, int S) {
    __shared__ int cnt[16];
    int mine = 0;
    // four samples per lane and round, their inputs loaded before any is decided
    // (the loads of a round overlap; every sample is read and written by one lane)
    constexpr int R = 4;
    for (int s0 = threadIdx.x; s0 < S; s0 += R * blockDim.x) {
        int act[R], cy[R];
        double rr[R], bn[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int s = s0 + u * int(blockDim.x);
            act[u] = s < S ? A.active[s] : 0;
            cy[u] = s < S ? A.cycles[2 * s + A.slot] : 0;
            rr[u] = s < S ? A.rr[s] : 0.0;
            bn[u] = s < S ? A.bnorm[s] : 1.0;
        }
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int s = s0 + u * int(blockDim.x);
            if (act[u] == 0) continue;
            const int cyc = cy[u] + A.inc;
            A.cycles[2 * s + A.slot] = cyc;
            const double rel = sqrt(rr[u]) / bn[u];
            bool stop = false;
            if (!isfinite(rel)) {
                A.flags[s] |= FMGMC_FLAG_NONFINITE;
                stop = true;
            } else if (rel <= A.tol) {
                stop = true;
            } else if (A.inc > 0 && cyc >= A.max_cycles) {
                A.flags[s] |= FMGMC_FLAG_NOTCONV;
                stop = true;
            }
            if (stop) {
                A.active[s] = 0;
                A.qout[s] = A.q[s];
            } else {
                ++mine;
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) mine += __shfl_xor(mine, o);
    if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < int(blockDim.x >> 6); ++w) t += cnt[w];
        A.n_active[0] = t;
    }
}

template <typename V>
__global__ void k_fill(V *p, V v, int64_t n) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

// ---- compensated sums: each lane sums a contiguous chunk in order (Neumaier),
// then the lanes' (sum, compensation) pairs are combined in a fixed tree.
struct NS {
    double s, c;
};
__device__ __forceinline__ void nadd(NS &a, double x) {
    const double t = a.s + x;
    a.c += (fabs(a.s) >= fabs(x)) ? (a.s - t) + x : (x - t) + a.s;
    a.s = t;
}
__device__ __forceinline__ NS ncomb(NS a, NS b) {
    nadd(a, b.s);
    a.c += b.c;
    return a;
}

constexpr int RT = 256;

template <typename Fn>
__device__ double block_nsum(int64_t n, Fn val, NS *sh) {
    const int64_t chunk = (n + RT - 1) / RT;
    const int64_t lo = threadIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    NS a{0.0, 0.0};
    for (int64_t k = lo; k < hi; ++k) nadd(a, val(k));
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int w = RT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] = ncomb(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    const double r = sh[0].s + sh[0].c;
    __syncthreads();
    return r;
}

// out: [mean_y, var_y, mean_qf, var_qf, mean_qc]; RQMC (nshift > 1): var_y is the
// variance of the estimate from the per-shift means, shift means in scratch.
__global__ __launch_bounds__(RT) void k_level_reduce(const double *qf, const double *qc, int64_t n, int nshift,
                                                     double *out, double *shift_means) {
    __shared__ NS sh[RT];
    if (nshift <= 1) {
        const double my = block_nsum(n, [&](int64_t k) { return qf[k] - qc[k]; }, sh) / double(n);
        const double mf = block_nsum(n, [&](int64_t k) { return qf[k]; }, sh) / double(n);
        const double mc = block_nsum(n, [&](int64_t k) { return qc[k]; }, sh) / double(n);
        const double vy = n > 1 ? block_nsum(n, [&](int64_t k) { const double d = (qf[k] - qc[k]) - my; return d * d; }, sh) / double(n - 1) : 0.0;
        const double vf = n > 1 ? block_nsum(n, [&](int64_t k) { const double d = qf[k] - mf; return d * d; }, sh) / double(n - 1) : 0.0;
        if (threadIdx.x == 0) {
            out[0] = my; out[1] = vy; out[2] = mf; out[3] = vf; out[4] = mc;
        }
        return;
    }
    const int64_t np = n / nshift;
    for (int r = 0; r < nshift; ++r) {
        const double *f = qf + size_t(r) * np, *c = qc + size_t(r) * np;
        const double m = block_nsum(np, [&](int64_t k) { return f[k] - c[k]; }, sh) / double(np);
        if (threadIdx.x == 0) shift_means[r] = m;
    }
    __syncthreads();
    const double m = block_nsum(nshift, [&](int64_t k) { return shift_means[k]; }, sh) / double(nshift);
    const double v = block_nsum(nshift, [&](int64_t k) { const double d = shift_means[k] - m; return d * d; }, sh) /
                     (double(nshift) * double(nshift - 1));
    const double mf = block_nsum(n, [&](int64_t k) { return qf[k]; }, sh) / double(n);
    const double mc = block_nsum(n, [&](int64_t k) { return qc[k]; }, sh) / double(n);
    const double vf = n > 1 ? block_nsum(n, [&](int64_t k) { const double d = qf[k] - mf; return d * d; }, sh) / double(n - 1) : 0.0;
    if (threadIdx.x == 0) {
        out[0] = m; out[1] = v; out[2] = mf; out[3] = vf; out[4] = mc;
    }
}

}  // namespace

int launch_ir(const IRArgs &a, int S, hipStream_t st) {
    if (a.n < 8 || a.n > 1024) {
        set_error("launch_ir: n out of range");
        return FMGMC_EINVAL;
    }
    if (S <= 0) return FMGMC_OK;
    const size_t lds = (6 * size_t(a.n) + 18) * sizeof(double);
    hipLaunchKernelGGL(k_ir, dim3(S), dim3(a.n), lds, st, a);
    return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP;
}

template <typename TS>
int launch_interp64(int n, const TS *xc, double *p, const int32_t *active, const Bnd &g, int S,
                    hipStream_t st) {
    if (S <= 0) return FMGMC_OK;
    dim3 grid((n * n / 4 + 255) / 256, S);
    hipLaunchKernelGGL(k_interp64<TS>, grid, dim3(256), 0, st, n, xc, p, active, g);
    return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP;
}
template int launch_interp64<float>(int, const float *, double *, const int32_t *, const Bnd &, int, hipStream_t);
template int launch_interp64<double>(int, const double *, double *, const int32_t *, const Bnd &, int, hipStream_t);

template <typename T>
int launch_bnorm(int n, const T *K, const Bnd &g, double *bn, int S, hipStream_t st) {
    if (S <= 0) return FMGMC_OK;
    hipLaunchKernelGGL(k_bnorm<T>, dim3(S), dim3(256), 0, st, n, K, g, bn);
    return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP;
}
template int launch_bnorm<double>(int, const double *, const Bnd &, double *, int, hipStream_t);
template int launch_bnorm<float>(int, const float *, const Bnd &, double *, int, hipStream_t);

int launch_check(const CheckArgs &a, int S, hipStream_t st) {
    if (S <= 0) return FMGMC_OK;
    hipLaunchKernelGGL(k_check, dim3(1), dim3(1024), 0, st, a, S);
    return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP;
}

int launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return FMGMC_OK;
    hipLaunchKernelGGL(k_fill<int32_t>, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
    return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP;
}
int launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return FMGMC_OK;
    hipLaunchKernelGGL(k_fill<uint8_t>, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
    return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP;
}
int launch_fill_f64(double *p, double v, int64_t n, hipStream_t st) {
    if (n <= 0) return FMGMC_OK;
    hipLaunchKernelGGL(k_fill<double>, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
    return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP;
}

int launch_level_reduce(const double *qf, const double *qc, int64_t n, int nshift, double *out,
                        double *shift_means, hipStream_t st) {
    if (n <= 0 || nshift < 1 || (nshift > 1 && n % nshift != 0)) {
        set_error("launch_level_reduce: bad sizes");
        return FMGMC_EINVAL;
    }
    hipLaunchKernelGGL(k_level_reduce, dim3(1), dim3(RT), 0, st, qf, qc, n, nshift, out, shift_means);
    return hipGetLastError() == hipSuccess ? FMGMC_OK : FMGMC_EHIP;
}


// Fixed device scratch of the allocation-free estimator entry point: slots
// 0..4 take a level's results, slots 8.. the per-shift means of RQMC. Each
// device holds its own copy until the process ends; its address is looked
// up once per device (with that device current) and kept, and host code
// only ever passes that address on.
__device__ __align__(256) double scratch[kEstScratchDoubles];

namespace {
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int estimate_scratch(double **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        set_error("estimate scratch: no current HIP device (or device index above the library's limit)");
        return FMGMC_EHIP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return FMGMC_EHIP;
        }
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return FMGMC_OK;
}

}  // namespace fmgmc
