// Host-side Karhunen-Loeve mode table of the separable exponential covariance
// (Section 3.1 (2) of the paper; the covariance is the nu = 1/2 Matern kernel
// applied per axis). Built once per context.
//
// 1-D: the eigenfunctions of exp(-c|s-t|) on [0,1] (c = 1/l) are
//   cos(w (s - 1/2)) with c cos(w/2) - w sin(w/2) = 0   (k even, 0-based)
//   sin(w (s - 1/2)) with w cos(w/2) + c sin(w/2) = 0   (k odd)
// with the k-th root in (k pi, (k+1) pi) and eigenvalue theta = 2c / (c^2 + w^2).
// 2-D: lambda_ab = sigma^2 theta_a theta_b; the M largest are kept, exact
// ties ordered by (a, b) ascending, a = mode along x.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace fmgmc {

namespace {

struct Char {
    double c;
    bool even;
    double f(double w) const {
        double h = 0.5 * w;
        return even ? c * std::cos(h) - w * std::sin(h) : w * std::cos(h) + c * std::sin(h);
    }
    double df(double w) const {
        double h = 0.5 * w, cs = std::cos(h), sn = std::sin(h);
        return even ? -0.5 * c * sn - sn - h * cs : cs - h * sn + 0.5 * c * cs;
    }
};

// Newton iteration kept inside a sign-change bracket; bisection when a step
// leaves it. Ends when the bracket holds no representable interior point.
double root_k(double c, int k) {
    Char g{c, (k % 2) == 0};
    double lo = k * M_PI, hi = (k + 1) * M_PI;
    double flo = g.f(lo);
    double w = 0.5 * (lo + hi);
    for (int it = 0; it < 300; ++it) {
        double fw = g.f(w);
        if (fw == 0.0) return w;
        if ((fw > 0.0) == (flo > 0.0)) {
            lo = w;
            flo = fw;
        } else {
            hi = w;
        }
        double mid = lo + 0.5 * (hi - lo);
        if (!(mid > lo && mid < hi)) break;
        double d = g.df(w);
        double nw = (d != 0.0) ? w - fw / d : mid;
        w = (nw > lo && nw < hi) ? nw : mid;
    }
    return std::fabs(g.f(lo)) <= std::fabs(g.f(hi)) ? lo : hi;
}

}  // namespace

int build_mode_table(double sigma2, double corr_len, int M, ModeTable &t) {
    if (!(sigma2 > 0.0) || !(corr_len > 0.0) || M < 1 || M > 4096) return FMGMC_EINVAL;
    const double c = 1.0 / corr_len;
    std::vector<double> w(M), th(M);
    for (int k = 0; k < M; ++k) {
        w[k] = root_k(c, k);
        th[k] = 2.0 * c / (c * c + w[k] * w[k]);
    }
    struct P { double lam; int32_t a, b; };
    std::vector<P> all;
    all.reserve(size_t(M) * M);
    for (int a = 0; a < M; ++a)
        for (int b = 0; b < M; ++b) all.push_back({sigma2 * (th[a] * th[b]), a, b});
    std::partial_sort(all.begin(), all.begin() + M, all.end(), [](const P &x, const P &y) {
        if (x.lam != y.lam) return x.lam > y.lam;
        if (x.a != y.a) return x.a < y.a;
        return x.b < y.b;
    });
    t.M = M;
    t.a.resize(M);
    t.b.resize(M);
    t.lam.resize(M);
    t.kmax = 0;
    for (int m = 0; m < M; ++m) {
        t.a[m] = all[m].a;
        t.b[m] = all[m].b;
        t.lam[m] = all[m].lam;
        t.kmax = std::max(t.kmax, std::max(all[m].a, all[m].b));
    }
    t.w.assign(w.begin(), w.begin() + (t.kmax + 1));
    return FMGMC_OK;
}

void tabulate_phi(const ModeTable &t, int n, std::vector<double> &tab) {
    const int nk = t.kmax + 1;
    tab.assign(size_t(nk) * n, 0.0);
    for (int k = 0; k < nk; ++k) {
        const double w = t.w[k];
        const bool even = (k % 2) == 0;
        const double nrm = 1.0 / std::sqrt(even ? 0.5 + std::sin(w) / (2.0 * w)
                                                : 0.5 - std::sin(w) / (2.0 * w));
        for (int i = 0; i < n; ++i) {
            const double s = double(i) / double(n) - 0.5;
            tab[size_t(k) * n + i] = (even ? std::cos(w * s) : std::sin(w * s)) * nrm;
        }
    }
}

}  // namespace fmgmc
