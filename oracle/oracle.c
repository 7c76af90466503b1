/*
 * Plain FP64 CPU oracle for the full-multigrid multilevel Monte Carlo method
 * for single-phase Darcy flow with a log-normal random permeability
 * (Liu, Li, Sun, Yu, arXiv:1910.04727).
 *
 * THIS IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT. Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it. It shares
 * no code, header or table with the HIP library; the two are built separately
 * and neither includes the other.
 *
 * Everything is written for clarity, in double precision, one sample at a
 * time, following the definitions in the order the paper states them:
 *   - model problem: Section 2.1, Eq. (1); Cases I and II of Table 1
 *     (Section 3.1). Case II: Dirichlet pressure on the west/east sides, no
 *     flow on north/south, QoI = outflow through the east side. Case I:
 *     Dirichlet pressure on all four sides, QoI = the pressure at the centre.
 *     Boundary values are passed in; the problem is linear, so the paper's
 *     values are a multiple of any scaled set (1/0 here for Case II).
 *   - discretisation: Section 3.1 (1), cell-centred finite volumes on a
 *     uniform n x n grid of the unit square, harmonic-mean face
 *     transmissibilities, half-cell transmissibility 2K on Dirichlet faces.
 *   - random field: Section 3.1 (2), Karhunen-Loeve expansion; the covariance
 *     used here is the separable exponential sigma^2 exp(-|dx|/l - |dy|/l)
 *     (the nu = 1/2 member of the Matern family of Eq. (Matern)), whose
 *     eigenpairs are products of the 1-D exponential-kernel eigenpairs.
 *   - coefficient coarsening: Section 2.5 (Coarsening), k^c_{I,J} = k^f of the
 *     first (lower-left) fine cell of the 2x2 block.
 *   - solver: Section 2.5 (Multigrid) and Algorithm 3 (FMG-MLMC): full
 *     multigrid; the coarse-mesh QoI Q^c_l is read from the FMG stage one grid
 *     below the finest, as a by-product of the pass that yields Q^f_l.
 *   - estimators: Section 2.1 Eqs. (2)-(5) and the estimator \hat Y_l;
 *     Section 2.3 (optimal N_l by a Lagrange multiplier); Section 2.4 (QMC).
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   field sampled at cell lower-left corners (i h, j h); V(nu1,nu2) cycles of
 *   red-black Gauss-Seidel (red = (i+j) even, red sweep first) whose
 *   coarse-grid corrections on grids of n <= 64 are W-cycles, residual
 *   restriction by summing the four children, bilinear cell-centred
 *   prolongation, stage operators rediscretised from the injected K and
 *   V-cycle correction operators by face averaging (see section 4),
 *   direct (Cholesky) solve on the coarsest grid, the two QoI stages driven
 *   to ||b - A p||_2 <= tol ||b||_2 and intermediate FMG stages given one
 *   V-cycle.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* 1. Karhunen-Loeve eigenpairs of exp(-c|s-t|) on [0,1]  (Section 3.1 (2))  */
/* ------------------------------------------------------------------------ */
/*
 * The integral equation  int_0^1 exp(-c|s-t|) phi(t) dt = theta phi(s)  turns
 * into phi'' + w^2 phi = 0 with theta = 2c/(c^2+w^2).  Centred at s = 1/2 the
 * solutions are cos(w (s-1/2)) (even) with c cos(w/2) = w sin(w/2), and
 * sin(w (s-1/2)) (odd) with w cos(w/2) = -c sin(w/2).  The n-th root (n >= 1)
 * lies in ((n-1) pi, n pi); odd n gives an even function, even n an odd one.
 */
static double kl_char(double c, int n, double w)
{
    if (n % 2 == 1)
        return c * cos(0.5 * w) - w * sin(0.5 * w);
    return w * cos(0.5 * w) + c * sin(0.5 * w);
}

/* n-th root (n >= 1) by bisection until the bracket cannot shrink. */
double oracle_kl_root(double c, int n)
{
    double lo = (n - 1) * M_PI, hi = n * M_PI;
    double flo = kl_char(c, n, lo);
    for (int it = 0; it < 400; ++it) {
        double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi))
            break;
        double fm = kl_char(c, n, mid);
        if (fm == 0.0)
            return mid;
        if ((fm > 0.0) == (flo > 0.0)) {
            lo = mid;
            flo = fm;
        } else {
            hi = mid;
        }
    }
    return 0.5 * (lo + hi);
}

double oracle_kl_theta(double c, double w) { return 2.0 * c / (c * c + w * w); }

/* Normalised eigenfunction number n (n >= 1) at s in [0,1]. */
double oracle_kl_phi(int n, double w, double s)
{
    if (n % 2 == 1)
        return cos(w * (s - 0.5)) / sqrt(0.5 + sin(w) / (2.0 * w));
    return sin(w * (s - 0.5)) / sqrt(0.5 - sin(w) / (2.0 * w));
}

/* First `count` 1-D roots and eigenvalues (index k = 0 is n = 1). */
void oracle_kl_1d(double corr_len, int count, double *w, double *theta)
{
    double c = 1.0 / corr_len;
    for (int k = 0; k < count; ++k) {
        w[k] = oracle_kl_root(c, k + 1);
        theta[k] = oracle_kl_theta(c, w[k]);
    }
}

typedef struct {
    double lam;
    int a, b;
} kl_pair;

/* Descending eigenvalue; exact ties broken by (a ascending, b ascending). */
static int kl_pair_cmp(const void *pa, const void *pb)
{
    const kl_pair *x = (const kl_pair *)pa, *y = (const kl_pair *)pb;
    if (x->lam > y->lam) return -1;
    if (x->lam < y->lam) return 1;
    if (x->a != y->a) return x->a < y->a ? -1 : 1;
    if (x->b != y->b) return x->b < y->b ? -1 : 1;
    return 0;
}

/*
 * 2-D separable table: lambda_{ab} = sigma2 * (theta_a * theta_b), a = x-mode,
 * b = y-mode (0-based).  Keeps the M largest.  Every kept pair has a, b < M
 * (the M pairs (a,0), a < M, all beat any pair with an index >= M), so the
 * candidate set is {0..M-1}^2.  Returns 0, or -1 on bad arguments / memory.
 */
int oracle_kl_table(double sigma2, double corr_len, int M, int *a, int *b, double *lam)
{
    if (M < 1 || !(corr_len > 0.0) || !(sigma2 >= 0.0))
        return -1;
    double *w = (double *)malloc(sizeof(double) * M);
    double *th = (double *)malloc(sizeof(double) * M);
    kl_pair *p = (kl_pair *)malloc(sizeof(kl_pair) * (size_t)M * M);
    if (!w || !th || !p) {
        free(w); free(th); free(p);
        return -1;
    }
    oracle_kl_1d(corr_len, M, w, th);
    size_t q = 0;
    for (int ia = 0; ia < M; ++ia)
        for (int ib = 0; ib < M; ++ib) {
            p[q].lam = sigma2 * (th[ia] * th[ib]);
            p[q].a = ia;
            p[q].b = ib;
            ++q;
        }
    qsort(p, q, sizeof(kl_pair), kl_pair_cmp);
    for (int m = 0; m < M; ++m) {
        a[m] = p[m].a;
        b[m] = p[m].b;
        lam[m] = p[m].lam;
    }
    free(w); free(th); free(p);
    return 0;
}

/*
 * Field on the n x n grid for one sample:
 *   g(x_i, y_j) = sum_m xi_m sqrt(lambda_m) phi_{a_m}(x_i) phi_{b_m}(y_j),
 *   K = exp(g),  x_i = i h, y_j = j h (cell lower-left corners), h = 1/n.
 * K is row-major [j][i] (x fastest).
 */
void oracle_field(int n, double corr_len, int M, const int *a, const int *b,
                  const double *lam, const double *xi, double *K)
{
    double c = 1.0 / corr_len, h = 1.0 / n;
    int kmax = 0;
    for (int m = 0; m < M; ++m) {
        if (a[m] > kmax) kmax = a[m];
        if (b[m] > kmax) kmax = b[m];
    }
    int nk = kmax + 1;
    double *tab = (double *)malloc(sizeof(double) * (size_t)nk * n);
    for (int k = 0; k < nk; ++k) {
        double w = oracle_kl_root(c, k + 1);
        for (int i = 0; i < n; ++i)
            tab[(size_t)k * n + i] = oracle_kl_phi(k + 1, w, i * h);
    }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            double g = 0.0;
            for (int m = 0; m < M; ++m)
                g += xi[m] * sqrt(lam[m]) * tab[(size_t)a[m] * n + i] * tab[(size_t)b[m] * n + j];
            K[(size_t)j * n + i] = exp(g);
        }
    free(tab);
}

/* Coarsening by injection (Section 2.5): Kc[J][I] = Kf[2J][2I]. */
void oracle_coarsen(int n, const double *Kf, double *Kc)
{
    int nc = n / 2;
    for (int J = 0; J < nc; ++J)
        for (int I = 0; I < nc; ++I)
            Kc[(size_t)J * nc + I] = Kf[(size_t)(2 * J) * n + 2 * I];
}

/* ------------------------------------------------------------------------ */
/* 2. Finite-volume operator (Section 3.1 (1), Cases I and II of Table 1)   */
/* ------------------------------------------------------------------------ */
/*
 * Boundary conditions (Table 1). `cs` selects the case:
 *   cs = 2 (Case II): Dirichlet on the west and east sides, no flow through
 *          the south and north sides; QoI = outflow through the east side;
 *   cs = 1 (Case I):  Dirichlet on all four sides; QoI = u(1/2, 1/2).
 * g[4] = Dirichlet values on the west, east, south and north sides (the
 * south/north entries are unused in Case II).
 */
static double harmonic(double k1, double k2) { return 2.0 * k1 * k2 / (k1 + k2); }

/*
 * Face transmissibilities of the integrated cell-centred scheme on square
 * cells (the h/h factor cancels):
 *   Tx[j][i], i = 0..n : face between cells i-1 and i of row j;
 *                        face 0 (west) and face n (east) are Dirichlet, 2K.
 *   Ty[j][i], j = 0..n : face between rows j-1 and j of column i;
 *                        faces 0 (south) and n (north) are no-flow, 0, in
 *                        Case II and Dirichlet, 2K, in Case I.
 * Layout: Tx has (n+1) entries per row, Ty has n entries per face row.
 */
void oracle_faces(int n, const double *K, int cs, double *Tx, double *Ty)
{
    for (int j = 0; j < n; ++j) {
        const double *Kr = K + (size_t)j * n;
        double *T = Tx + (size_t)j * (n + 1);
        T[0] = 2.0 * Kr[0];
        for (int i = 1; i < n; ++i)
            T[i] = harmonic(Kr[i - 1], Kr[i]);
        T[n] = 2.0 * Kr[n - 1];
    }
    for (int i = 0; i < n; ++i) {
        Ty[i] = (cs == 1) ? 2.0 * K[i] : 0.0;
        Ty[(size_t)n * n + i] = (cs == 1) ? 2.0 * K[(size_t)(n - 1) * n + i] : 0.0;
    }
    for (int j = 1; j < n; ++j)
        for (int i = 0; i < n; ++i)
            Ty[(size_t)j * n + i] = harmonic(K[(size_t)(j - 1) * n + i], K[(size_t)j * n + i]);
}

/* Diagonal D_P = sum of the four face transmissibilities of cell (i,j). */
static double diag_of(int n, const double *Tx, const double *Ty, int i, int j)
{
    return Tx[(size_t)j * (n + 1) + i] + Tx[(size_t)j * (n + 1) + i + 1]
         + Ty[(size_t)j * n + i] + Ty[(size_t)(j + 1) * n + i];
}

/* Sum over interior neighbours of T_nb * x_nb for cell (i,j). */
static double offdiag_sum(int n, const double *Tx, const double *Ty, const double *x, int i, int j)
{
    size_t P = (size_t)j * n + i;
    double s = 0.0;
    if (i > 0) s += Tx[(size_t)j * (n + 1) + i] * x[P - 1];
    if (i < n - 1) s += Tx[(size_t)j * (n + 1) + i + 1] * x[P + 1];
    if (j > 0) s += Ty[(size_t)j * n + i] * x[P - n];
    if (j < n - 1) s += Ty[(size_t)(j + 1) * n + i] * x[P + n];
    return s;
}

/* y = A x : (A x)_P = D_P x_P - sum_nb T_nb x_nb. */
void oracle_apply(int n, const double *Tx, const double *Ty, const double *x, double *y)
{
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            size_t P = (size_t)j * n + i;
            y[P] = diag_of(n, Tx, Ty, i, j) * x[P] - offdiag_sum(n, Tx, Ty, x, i, j);
        }
}

/* Right-hand side: Dirichlet data enters through the boundary faces that carry it. */
void oracle_rhs(int n, const double *Tx, const double *Ty, const double *g, int cs, double *b)
{
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            double v = 0.0;
            if (i == 0) v += Tx[(size_t)j * (n + 1)] * g[0];
            if (i == n - 1) v += Tx[(size_t)j * (n + 1) + n] * g[1];
            if (cs == 1 && j == 0) v += Ty[i] * g[2];
            if (cs == 1 && j == n - 1) v += Ty[(size_t)n * n + i] * g[3];
            b[(size_t)j * n + i] = v;
        }
}

/* r = b - A x */
void oracle_residual(int n, const double *Tx, const double *Ty, const double *b,
                     const double *x, double *r)
{
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            size_t P = (size_t)j * n + i;
            r[P] = b[P] - (diag_of(n, Tx, Ty, i, j) * x[P] - offdiag_sum(n, Tx, Ty, x, i, j));
        }
}

/*
 * QoI of Table 1.
 * Case II: outflow through the east side, sum_j T_east (p_{n-1,j} - pE).
 * Case I: u(1/2, 1/2). For even n the point is the corner shared by the four
 * centre cells, and the bilinear interpolant of the cell values there is
 * their mean.
 */
double oracle_qoi(int n, const double *Tx, const double *x, const double *g, int cs)
{
    if (cs == 1) {
        int c = n / 2;
        return 0.25 * (x[(size_t)(c - 1) * n + c - 1] + x[(size_t)(c - 1) * n + c]
                       + x[(size_t)c * n + c - 1] + x[(size_t)c * n + c]);
    }
    double q = 0.0;
    for (int j = 0; j < n; ++j)
        q += Tx[(size_t)j * (n + 1) + n] * (x[(size_t)j * n + n - 1] - g[1]);
    return q;
}

double oracle_norm2(size_t len, const double *v)
{
    double s = 0.0;
    for (size_t k = 0; k < len; ++k)
        s += v[k] * v[k];
    return sqrt(s);
}

/* ------------------------------------------------------------------------ */
/* 3. Multigrid components                                                   */
/* ------------------------------------------------------------------------ */

/* One half-sweep of Gauss-Seidel over the cells with (i+j) % 2 == colour. */
void oracle_rbgs_half(int n, const double *Tx, const double *Ty, const double *b,
                      double *x, int colour)
{
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            if ((i + j) % 2 != colour)
                continue;
            size_t P = (size_t)j * n + i;
            x[P] = (b[P] + offdiag_sum(n, Tx, Ty, x, i, j)) / diag_of(n, Tx, Ty, i, j);
        }
}

/* Restriction of an integrated residual: the coarse cell gets the sum of its four children. */
void oracle_restrict(int n, const double *r, double *rc)
{
    int nc = n / 2;
    for (int J = 0; J < nc; ++J)
        for (int I = 0; I < nc; ++I) {
            size_t f = (size_t)(2 * J) * n + 2 * I;
            rc[(size_t)J * nc + I] = r[f] + r[f + 1] + r[f + n] + r[f + n + 1];
        }
}

/*
 * Value of a coarse-grid function outside the grid, for bilinear
 * interpolation. A Dirichlet side with value g reflects oddly about it,
 * 2 g - value; a no-flow side mirrors the adjacent cell. g is 0 for a
 * correction and the boundary data for a solution. Outside in both
 * directions (a corner), the south/north rule is applied first and the
 * west/east rule to its result.
 */
static double ghost_row(int nc, const double *v, int I, int J, const double *g, int cs)
{
    if (J >= 0 && J < nc)
        return v[(size_t)J * nc + I];
    int Jc = J < 0 ? 0 : nc - 1;
    if (cs == 1)
        return 2.0 * (J < 0 ? g[2] : g[3]) - v[(size_t)Jc * nc + I];
    return v[(size_t)Jc * nc + I];
}

static double ghosted(int nc, const double *v, int I, int J, const double *g, int cs)
{
    if (I < 0) return 2.0 * g[0] - ghost_row(nc, v, 0, J, g, cs);
    if (I >= nc) return 2.0 * g[1] - ghost_row(nc, v, nc - 1, J, g, cs);
    return ghost_row(nc, v, I, J, g, cs);
}

/* Bilinear cell-centred interpolation at fine cell (i,j): weights 9,3,3,1 / 16. */
static double bilinear(int nc, const double *v, int i, int j, const double *g, int cs)
{
    int I = i / 2, J = j / 2;
    int di = (i % 2) ? 1 : -1, dj = (j % 2) ? 1 : -1;
    return (9.0 * ghosted(nc, v, I, J, g, cs) + 3.0 * ghosted(nc, v, I + di, J, g, cs)
            + 3.0 * ghosted(nc, v, I, J + dj, g, cs) + ghosted(nc, v, I + di, J + dj, g, cs))
           / 16.0;
}

/* x (fine, n = 2 nc) += P ec, homogeneous boundary data. */
void oracle_prolong_add(int nc, const double *ec, int cs, double *x)
{
    static const double zero[4] = {0.0, 0.0, 0.0, 0.0};
    int n = 2 * nc;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
            x[(size_t)j * n + i] += bilinear(nc, ec, i, j, zero, cs);
}

/* FMG interpolation of a solution: x (fine) = P xc with the Dirichlet data g. */
void oracle_fmg_interp(int nc, const double *xc, const double *g, int cs, double *x)
{
    int n = 2 * nc;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
            x[(size_t)j * n + i] = bilinear(nc, xc, i, j, g, cs);
}

/* Dense Cholesky A = L L^T of the N = n*n coarsest operator (lower triangle in L). */
int oracle_chol_factor(int n, const double *Tx, const double *Ty, double *L)
{
    int N = n * n;
    double *A = L;
    memset(A, 0, sizeof(double) * (size_t)N * N);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            int P = j * n + i;
            A[(size_t)P * N + P] = diag_of(n, Tx, Ty, i, j);
            if (i > 0) A[(size_t)P * N + P - 1] = -Tx[(size_t)j * (n + 1) + i];
            if (i < n - 1) A[(size_t)P * N + P + 1] = -Tx[(size_t)j * (n + 1) + i + 1];
            if (j > 0) A[(size_t)P * N + P - n] = -Ty[(size_t)j * n + i];
            if (j < n - 1) A[(size_t)P * N + P + n] = -Ty[(size_t)(j + 1) * n + i];
        }
    for (int c = 0; c < N; ++c) {
        double d = A[(size_t)c * N + c];
        for (int k = 0; k < c; ++k)
            d -= L[(size_t)c * N + k] * L[(size_t)c * N + k];
        if (!(d > 0.0))
            return -1;
        d = sqrt(d);
        L[(size_t)c * N + c] = d;
        for (int r = c + 1; r < N; ++r) {
            double s = A[(size_t)r * N + c];
            for (int k = 0; k < c; ++k)
                s -= L[(size_t)r * N + k] * L[(size_t)c * N + k];
            L[(size_t)r * N + c] = s / d;
        }
    }
    return 0;
}

void oracle_chol_solve(int N, const double *L, const double *b, double *x)
{
    for (int r = 0; r < N; ++r) {
        double s = b[r];
        for (int k = 0; k < r; ++k)
            s -= L[(size_t)r * N + k] * x[k];
        x[r] = s / L[(size_t)r * N + r];
    }
    for (int r = N - 1; r >= 0; --r) {
        double s = x[r];
        for (int k = r + 1; k < N; ++k)
            s -= L[(size_t)k * N + r] * x[k];
        x[r] = s / L[(size_t)r * N + r];
    }
}

/* ------------------------------------------------------------------------ */
/* 4. Hierarchy, V-cycle and full multigrid (Section 2.5, Algorithm 3)       */
/* ------------------------------------------------------------------------ */
/*
 * Two kinds of operators live on each grid:
 *   - the STAGE operator A^(n): rediscretised from the injected field K^(n);
 *     it defines the discrete problem whose solution gives the QoI of that
 *     grid (this is what makes Q^c_l and Q^f_{l-1} the same discrete quantity);
 *   - CORRECTION operators, used only inside V-cycles below the stage being
 *     solved: each coarse face transmissibility is the mean of the two fine
 *     faces that make it up (per row pair for x-faces, per column pair for
 *     y-faces), applied recursively from the stage operator downward. This is
 *     the transmissibility of the two fine half-paths in series, summed over
 *     the two parallel rows, and stays an SPD M-matrix. It changes how fast
 *     the cycles converge, never the converged solution.
 * Correction pyramids are built from the operator of each QoI stage (the
 * coarse-mesh stage n_f/2 on levels >= 1, and the fine stage n_f); stages
 * below n_f/2 use the pyramid of n_f/2 (of n_f on level 0).
 */
typedef struct {
    int n;
    double *Tx, *Ty;   /* faces, layouts as in oracle_faces */
} oop;

typedef struct {
    int n;
    double *x, *b, *r; /* correction, its right-hand side, residual scratch */
} oscratch;

static void op_alloc(oop *o, int n)
{
    o->n = n;
    o->Tx = (double *)calloc((size_t)n * (n + 1), sizeof(double));
    o->Ty = (double *)calloc((size_t)(n + 1) * n, sizeof(double));
}

static void op_free(oop *o)
{
    free(o->Tx);
    free(o->Ty);
    o->Tx = o->Ty = NULL;
}

/* Correction operator on n/2 from operator F on n: mean of the two fine faces. */
void oracle_coarsen_faces(int n, const double *Txf, const double *Tyf, double *Txc, double *Tyc)
{
    int nc = n / 2;
    for (int J = 0; J < nc; ++J)
        for (int I = 0; I <= nc; ++I)
            Txc[(size_t)J * (nc + 1) + I] = 0.5 * (Txf[(size_t)(2 * J) * (n + 1) + 2 * I]
                                                  + Txf[(size_t)(2 * J + 1) * (n + 1) + 2 * I]);
    for (int J = 0; J <= nc; ++J)
        for (int I = 0; I < nc; ++I)
            Tyc[(size_t)J * nc + I] = 0.5 * (Tyf[(size_t)(2 * J) * n + 2 * I]
                                            + Tyf[(size_t)(2 * J) * n + 2 * I + 1]);
}

/* A cycle context: ops[0..top], ops[top] the operator being solved. */
typedef struct {
    const oop *ops;
    oscratch *s;
    const double *chol; /* Cholesky factor of ops[0] */
    int nu1, nu2;
    int wmax;           /* coarse grids with n <= wmax are cycled twice (W-cycle) */
    int cs;             /* boundary case (section 2 above) */
} ovc;

/*
 * One multigrid cycle for ops[k] x = b (x updated in place): nu1 red-black
 * sweeps, residual restricted to the next coarser grid, coarse-grid
 * correction from zero, bilinear prolongation, nu2 sweeps. The coarse-grid
 * correction is itself one cycle, or two in succession when the coarse grid
 * has n <= wmax and is not the coarsest (a W-cycle below that size, a
 * V(nu1,nu2) cycle above it); the coarsest grid is solved directly.
 */
static void vcycle(const ovc *V, int k, double *x, const double *b)
{
    const oop *A = &V->ops[k];
    int n = A->n;
    if (k == 0) {
        oracle_chol_solve(n * n, V->chol, b, x);
        return;
    }
    for (int s = 0; s < V->nu1; ++s) {
        oracle_rbgs_half(n, A->Tx, A->Ty, b, x, 0);
        oracle_rbgs_half(n, A->Tx, A->Ty, b, x, 1);
    }
    oscratch *C = &V->s[k - 1];
    oracle_residual(n, A->Tx, A->Ty, b, x, V->s[k].r);
    oracle_restrict(n, V->s[k].r, C->b);
    memset(C->x, 0, sizeof(double) * (size_t)C->n * C->n);
    vcycle(V, k - 1, C->x, C->b);
    if (C->n <= V->wmax && k - 1 > 0)
        vcycle(V, k - 1, C->x, C->b);
    oracle_prolong_add(C->n, C->x, V->cs, x);
    for (int s = 0; s < V->nu2; ++s) {
        oracle_rbgs_half(n, A->Tx, A->Ty, b, x, 0);
        oracle_rbgs_half(n, A->Tx, A->Ty, b, x, 1);
    }
}

/* Relative residual ||b - A x||_2 / ||b||_2. */
static double relres(const oop *A, double *r, const double *x, const double *b)
{
    size_t N = (size_t)A->n * A->n;
    oracle_residual(A->n, A->Tx, A->Ty, b, x, r);
    return oracle_norm2(N, r) / oracle_norm2(N, b);
}

/*
 * Full multigrid pass for one sample on MLMC level `level` (Algorithm 3):
 * K_fine is the n_fine x n_fine field. The stage on n_fine/2 yields Q^c
 * (level >= 1; Q^c = 0 on level 0) and the stage on n_fine yields Q^f. Both
 * are driven to ||b - A p|| <= tol ||b|| (at most max_cycles V-cycles, at
 * least one); intermediate stages get one V-cycle; the coarsest stage is
 * solved directly.
 *
 * cycles[0], cycles[1] = V-cycles spent at the coarse / fine QoI stage.
 * flags: bit0 = a QoI stage did not reach tol, bit1 = non-finite residual.
 * hist (optional, 2*max_cycles): relative residual after each cycle at the
 * coarse (first half) and fine (second half) QoI stage; unused slots are -1.
 * Returns 0, or -1 if the grids do not fit (level >= 1 needs n_fine >=
 * 2 n_coarsest). A coarsest operator that is not positive definite (a
 * non-finite field) is reported through flags bit1.
 */
int oracle_fmg_sample(int n_fine, int n_coarsest, int level, const double *K_fine,
                      const double *g, int cs, double tol, int max_cycles, int nu1, int nu2,
                      int wmax, double *qf, double *qc, int *cycles, int *flags, double *hist)
{
    *qf = 0.0;
    *qc = 0.0;
    cycles[0] = cycles[1] = 0;
    *flags = 0;
    /* level >= 1 needs the coarse-mesh stage n_fine/2 inside the hierarchy */
    if (n_coarsest < 1 || n_fine < n_coarsest || (level >= 1 && n_fine < 2 * n_coarsest))
        return -1;
    int nlev = 1;
    for (int n = n_fine; n > n_coarsest; n /= 2)
        ++nlev;
    int top = nlev - 1;
    *qf = 0.0;
    *qc = 0.0;
    cycles[0] = cycles[1] = 0;
    *flags = 0;
    if (hist)
        for (int c = 0; c < 2 * max_cycles; ++c)
            hist[c] = -1.0;

    /* stage operators from the injected pyramid */
    oop *stage = (oop *)calloc(nlev, sizeof(oop));
    double **K = (double **)calloc(nlev, sizeof(double *));
    oscratch *S = (oscratch *)calloc(nlev, sizeof(oscratch));
    for (int k = top, n = n_fine; k >= 0; --k, n /= 2) {
        K[k] = (double *)malloc(sizeof(double) * (size_t)n * n);
        if (k == top)
            memcpy(K[k], K_fine, sizeof(double) * (size_t)n * n);
        else
            oracle_coarsen(2 * n, K[k + 1], K[k]);
        op_alloc(&stage[k], n);
        oracle_faces(n, K[k], cs, stage[k].Tx, stage[k].Ty);
        S[k].n = n;
        S[k].x = (double *)calloc((size_t)n * n, sizeof(double));
        S[k].b = (double *)calloc((size_t)n * n, sizeof(double));
        S[k].r = (double *)calloc((size_t)n * n, sizeof(double));
    }
    /* correction pyramids of the fine (index 1) and coarse (index 0) QoI stage */
    oop *pyr[2];
    int pyr_top[2] = {top - 1, top};
    int N0 = n_coarsest * n_coarsest;
    double *chol_stage = (double *)malloc(sizeof(double) * (size_t)N0 * N0);
    double *chol_pyr[2];
    int rc = oracle_chol_factor(n_coarsest, stage[0].Tx, stage[0].Ty, chol_stage);
    for (int q = 0; q < 2; ++q) {
        pyr[q] = (oop *)calloc(nlev, sizeof(oop));
        chol_pyr[q] = (double *)malloc(sizeof(double) * (size_t)N0 * N0);
        int t = pyr_top[q];
        if (t < 1)
            continue;
        for (int k = t - 1; k >= 0; --k) {
            op_alloc(&pyr[q][k], stage[k].n);
            const oop *F = (k == t - 1) ? &stage[t] : &pyr[q][k + 1];
            oracle_coarsen_faces(F->n, F->Tx, F->Ty, pyr[q][k].Tx, pyr[q][k].Ty);
        }
        rc |= oracle_chol_factor(n_coarsest, pyr[q][0].Tx, pyr[q][0].Ty, chol_pyr[q]);
    }
    if (rc != 0) {
        *flags = 2;
    } else {
        size_t Nmax = (size_t)n_fine * n_fine;
        double *p = (double *)calloc(Nmax, sizeof(double));
        double *pprev = (double *)calloc(Nmax, sizeof(double));
        double *bs = (double *)calloc(Nmax, sizeof(double));
        oop *ops = (oop *)calloc(nlev, sizeof(oop));
        for (int k = 0; k <= top; ++k) {
            const oop *A = &stage[k];
            oracle_rhs(A->n, A->Tx, A->Ty, g, cs, bs);
            if (k == 0)
                memset(p, 0, sizeof(double) * (size_t)A->n * A->n);
            else
                oracle_fmg_interp(stage[k - 1].n, pprev, g, cs, p);

            int is_fine = (k == top);
            int is_coarse = (level >= 1 && k == top - 1);
            int q = (level >= 1 && k <= top - 1) ? 0 : 1;
            ovc V;
            for (int j = 0; j < k; ++j)
                ops[j] = pyr[q][j];
            ops[k] = *A;
            V.ops = ops;
            V.s = S;
            V.chol = (k == 0) ? chol_stage : chol_pyr[q];
            V.nu1 = nu1;
            V.nu2 = nu2;
            V.wmax = wmax;
            V.cs = cs;

            if (is_fine || is_coarse) {
                int slot = is_fine ? 1 : 0;
                int ncyc = 0;
                double rel;
                if (k == 0) {
                    vcycle(&V, 0, p, bs); /* exact solve, no cycles */
                    rel = relres(A, S[0].r, p, bs);
                } else {
                    do {
                        vcycle(&V, k, p, bs);
                        ++ncyc;
                        rel = relres(A, S[k].r, p, bs);
                        if (hist)
                            hist[slot * max_cycles + ncyc - 1] = rel;
                        if (!isfinite(rel))
                            break;
                    } while (rel > tol && ncyc < max_cycles);
                }
                cycles[slot] = ncyc;
                if (!isfinite(rel))
                    *flags |= 2;
                else if (rel > tol && k > 0)
                    *flags |= 1;
                double qv = oracle_qoi(A->n, A->Tx, p, g, cs);
                if (is_fine)
                    *qf = qv;
                else
                    *qc = qv;
            } else {
                vcycle(&V, k, p, bs);
            }
            double *t = p;
            p = pprev;
            pprev = t;
        }
        free(p); free(pprev); free(bs); free(ops);
    }
    for (int k = 0; k < nlev; ++k) {
        free(K[k]);
        op_free(&stage[k]);
        free(S[k].x); free(S[k].b); free(S[k].r);
        op_free(&pyr[0][k]);
        op_free(&pyr[1][k]);
    }
    free(K); free(stage); free(S);
    free(pyr[0]); free(pyr[1]);
    free(chol_stage); free(chol_pyr[0]); free(chol_pyr[1]);
    return 0; /* a failed factorisation is a property of the sample: flagged above */
}

/*
 * Batched level solve: for each sample s, K = field(xi[s]) on n_fine, then one
 * FMG pass. xi is [ns][M] row-major. cycles is [ns][2]. OpenMP over samples
 * (nthreads <= 0: the runtime default).
 */
int oracle_solve_level(double sigma2, double corr_len, int M, const int *a, const int *b,
                       const double *lam, int n_fine, int n_coarsest, int level,
                       int64_t ns, const double *xi, const double *g, int cs, double tol,
                       int max_cycles, int nu1, int nu2, int wmax, double *qf, double *qc,
                       int *cycles, int *flags, int nthreads)
{
    (void)sigma2;
    int err = 0;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int64_t s = 0; s < ns; ++s) {
        double *K = (double *)malloc(sizeof(double) * (size_t)n_fine * n_fine);
        oracle_field(n_fine, corr_len, M, a, b, lam, xi + (size_t)s * M, K);
        int r = oracle_fmg_sample(n_fine, n_coarsest, level, K, g, cs, tol, max_cycles,
                                  nu1, nu2, wmax, &qf[s], &qc[s], &cycles[2 * s], &flags[s], NULL);
        if (r != 0)
            err |= 1;
        free(K);
    }
    return err ? -1 : 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* 5. Estimators (Section 2.1 Eqs. (2)-(5); Section 2.3; Section 2.4)        */
/* ------------------------------------------------------------------------ */

/* Neumaier-compensated sum in index order. */
double oracle_sum(int64_t n, const double *v)
{
    double s = 0.0, c = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double t = s + v[k];
        if (fabs(s) >= fabs(v[k]))
            c += (s - t) + v[k];
        else
            c += (v[k] - t) + s;
        s = t;
    }
    return s + c;
}

/*
 * Per-level Monte Carlo statistics of Y = Q^f - Q^c:
 * out[0] = mean Y, out[1] = sample variance of Y (two-pass, N-1),
 * out[2] = mean Q^f, out[3] = variance of Q^f, out[4] = mean Q^c.
 */
int oracle_level_stats(int64_t n, const double *qf, const double *qc, double *out)
{
    if (n < 1) return -1;
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    double *d = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t k = 0; k < n; ++k)
        y[k] = qf[k] - qc[k];
    double my = oracle_sum(n, y) / (double)n;
    for (int64_t k = 0; k < n; ++k)
        d[k] = (y[k] - my) * (y[k] - my);
    double vy = n > 1 ? oracle_sum(n, d) / (double)(n - 1) : 0.0;
    double mf = oracle_sum(n, qf) / (double)n;
    for (int64_t k = 0; k < n; ++k)
        d[k] = (qf[k] - mf) * (qf[k] - mf);
    double vf = n > 1 ? oracle_sum(n, d) / (double)(n - 1) : 0.0;
    double mc = oracle_sum(n, qc) / (double)n;
    out[0] = my; out[1] = vy; out[2] = mf; out[3] = vf; out[4] = mc;
    free(y); free(d);
    return 0;
}

/*
 * Randomised QMC level statistics: samples are grouped shift-major,
 * [nshift][npts]. For each shift r the level mean of Y over its points;
 * the estimate is the mean over shifts and its variance is
 * sum_r (Ybar_r - Ybar)^2 / (R (R-1)).  out[0] = estimate, out[1] = variance
 * of the estimate; shift_means (optional, R entries) receives Ybar_r.
 */
int oracle_rqmc_stats(int64_t npts, int nshift, const double *qf, const double *qc,
                      double *out, double *shift_means)
{
    if (npts < 1 || nshift < 1) return -1;
    double *y = (double *)malloc(sizeof(double) * (size_t)npts);
    double *mr = (double *)malloc(sizeof(double) * (size_t)nshift);
    for (int r = 0; r < nshift; ++r) {
        for (int64_t k = 0; k < npts; ++k)
            y[k] = qf[(size_t)r * npts + k] - qc[(size_t)r * npts + k];
        mr[r] = oracle_sum(npts, y) / (double)npts;
        if (shift_means) shift_means[r] = mr[r];
    }
    double m = oracle_sum(nshift, mr) / (double)nshift;
    double v = 0.0;
    if (nshift > 1) {
        double *d = (double *)malloc(sizeof(double) * (size_t)nshift);
        for (int r = 0; r < nshift; ++r)
            d[r] = (mr[r] - m) * (mr[r] - m);
        v = oracle_sum(nshift, d) / ((double)nshift * (nshift - 1));
        free(d);
    }
    out[0] = m;
    out[1] = v;
    free(y); free(mr);
    return 0;
}

/*
 * Optimal sample counts (Section 2.3): minimise sum_l N_l C_l subject to
 * sum_l V_l / N_l = eps^2 / 2.  A Lagrange multiplier gives
 * N_l = 2 eps^-2 sqrt(V_l / C_l) sum_k sqrt(V_k C_k), rounded up.
 */
void oracle_optimal_nl(int nlev, const double *V, const double *C, double eps, int64_t *N)
{
    double s = 0.0;
    for (int k = 0; k < nlev; ++k)
        s += sqrt(V[k] * C[k]);
    for (int l = 0; l < nlev; ++l)
        N[l] = (int64_t)ceil(2.0 / (eps * eps) * sqrt(V[l] / C[l]) * s);
}
