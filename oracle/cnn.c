/*
 * Plain FP64 CPU oracle of the learned warm start: a small residual
 * convolutional network that maps (log K, normalised FMG residual) on a stage
 * grid to a correction of the FMG start. The paper has no network; its
 * Section 2.5 defines the FMG pass whose start this corrects, and the pass
 * still iterates every sample to the same tolerance, so the estimator does not
 * depend on the network.
 *
 * THIS IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT (same rules as
 * oracle.c): it shares no code with the HIP library.
 *
 * Network (one sample; images [channel][row y][column x], x fastest):
 *   conv(a, W)[o][y][x] = sum_c sum_{dy,dx in -1..1} W[o][c][dy+1][dx+1] a[c][y+dy][x+dx],
 *     with a = 0 outside the n x n grid (zero padding, cross-correlation);
 *   z0 = conv(x, W0) + b0,          h0 = relu(z0)              (C_in -> F)
 *   zk = conv(h_{k-1}, Wk) + bk,    hk = h_{k-1} + relu(zk)    (F -> F), k = 1..R
 *   y  = conv(hR, Wo) + bo                                      (F -> 1)
 * Parameters, flattened in this order: W0 [F][C_in][3][3], b0 [F], then for
 * k = 1..R: Wk [F][F][3][3], bk [F], then Wo [1][F][3][3], bo [1].
 * Losses over a batch of B samples:
 *   error loss     L = (1 / (B n^2)) sum (y - t)^2 for targets t;
 *   residual loss  L = (1 / (B n^2)) sum (x1 - A y)^2, where A is the stage
 *     operator of Section 3.1 (1) (harmonic faces, 2K on the Dirichlet faces,
 *     homogeneous boundary data) built from K = exp(x0). With x1 = r / rms(r)
 *     and the start p~ + rms(r) y, x1 - A y is the normalised residual of the
 *     corrected start, the quantity the FMG stopping rule measures.
 * Optimiser: Adam (Kingma and Ba, 2015) with bias correction.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int64_t oracle_cnn_nparams(int cin, int F, int R)
{
    return (int64_t)F * cin * 9 + F + (int64_t)R * (F * F * 9 + F) + F * 9 + 1;
}

/* out[o] = b[o] + conv(a, W)[o], o < co; a has ci channels; n x n images */
static void conv3(int n, int ci, int co, const double *W, const double *b, const double *a, double *out)
{
    for (int o = 0; o < co; ++o)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                double s = b ? b[o] : 0.0;
                for (int c = 0; c < ci; ++c)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            const int yy = y + dy, xx = x + dx;
                            if (yy < 0 || yy >= n || xx < 0 || xx >= n) continue;
                            s += W[((o * ci + c) * 3 + dy + 1) * 3 + dx + 1] * a[((size_t)c * n + yy) * n + xx];
                        }
                out[((size_t)o * n + y) * n + x] = s;
            }
}

/* transposed convolution: g_a[c] += sum_o sum_taps W[o][c][tap] g[o][at the shifted cell] */
static void conv3_t(int n, int ci, int co, const double *W, const double *g, double *ga)
{
    for (int c = 0; c < ci; ++c)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                double s = 0.0;
                /* a[c][y][x] fed output (o, y - dy, x - dx) through tap (dy, dx) */
                for (int o = 0; o < co; ++o)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            const int yo = y - dy, xo = x - dx;
                            if (yo < 0 || yo >= n || xo < 0 || xo >= n) continue;
                            s += W[((o * ci + c) * 3 + dy + 1) * 3 + dx + 1] * g[((size_t)o * n + yo) * n + xo];
                        }
                ga[((size_t)c * n + y) * n + x] += s;
            }
}

/* weight and bias gradients: gW[o][c][tap] += sum_cells g[o][cell] a[c][cell + tap] */
static void conv3_w(int n, int ci, int co, const double *g, const double *a, double *gW, double *gb)
{
    for (int o = 0; o < co; ++o) {
        for (int c = 0; c < ci; ++c)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    double s = 0.0;
                    for (int y = 0; y < n; ++y)
                        for (int x = 0; x < n; ++x) {
                            const int yy = y + dy, xx = x + dx;
                            if (yy < 0 || yy >= n || xx < 0 || xx >= n) continue;
                            s += g[((size_t)o * n + y) * n + x] * a[((size_t)c * n + yy) * n + xx];
                        }
                    gW[((o * ci + c) * 3 + dy + 1) * 3 + dx + 1] += s;
                }
        double s = 0.0;
        for (size_t k = 0; k < (size_t)n * n; ++k) s += g[(size_t)o * n * n + k];
        gb[o] += s;
    }
}

/* Forward pass of B samples. x [B][cin][n][n], y [B][n][n]. If z and h are
 * non-NULL they receive the pre-activations and activations of the R + 1
 * hidden layers, [B][R+1][F][n][n] each. */
void oracle_cnn_forward(int n, int B, int cin, int F, int R, const double *theta, const double *x, double *y,
                        double *z, double *h)
{
    const size_t N = (size_t)n * n;
    double *zz = malloc(sizeof(double) * (R + 1) * F * N);
    double *hh = malloc(sizeof(double) * (R + 1) * F * N);
    for (int s = 0; s < B; ++s) {
        const double *p = theta;
        conv3(n, cin, F, p, p + F * cin * 9, x + (size_t)s * cin * N, zz);
        p += F * cin * 9 + F;
        for (size_t k = 0; k < F * N; ++k) hh[k] = zz[k] > 0.0 ? zz[k] : 0.0;
        for (int l = 1; l <= R; ++l) {
            double *zl = zz + (size_t)l * F * N, *hl = hh + (size_t)l * F * N;
            const double *hp = hh + (size_t)(l - 1) * F * N;
            conv3(n, F, F, p, p + F * F * 9, hp, zl);
            p += F * F * 9 + F;
            for (size_t k = 0; k < F * N; ++k) hl[k] = hp[k] + (zl[k] > 0.0 ? zl[k] : 0.0);
        }
        conv3(n, F, 1, p, p + F * 9, hh + (size_t)R * F * N, y + (size_t)s * N);
        if (z) memcpy(z + (size_t)s * (R + 1) * F * N, zz, sizeof(double) * (R + 1) * F * N);
        if (h) memcpy(h + (size_t)s * (R + 1) * F * N, hh, sizeof(double) * (R + 1) * F * N);
    }
    free(zz);
    free(hh);
}

/* FV operator of oracle.c (pinned by its closed forms) */
void oracle_faces(int n, const double *K, int cs, double *Tx, double *Ty);
void oracle_apply(int n, const double *Tx, const double *Ty, const double *x, double *y);

/* Loss and its gradient with respect to the parameters (grad, same layout as
 * theta): kind 0 = error loss with targets t [B][n][n], kind 1 = residual loss
 * (t unused). Returns L. */
double oracle_cnn_loss_grad_kind(int n, int B, int cin, int F, int R, const double *theta, const double *x,
                                 const double *t, int kind, double *grad)
{
    const size_t N = (size_t)n * n;
    const int64_t np = oracle_cnn_nparams(cin, F, R);
    double *y = malloc(sizeof(double) * N);
    double *z = malloc(sizeof(double) * (R + 1) * F * N);
    double *h = malloc(sizeof(double) * (R + 1) * F * N);
    double *gh = malloc(sizeof(double) * F * N);
    double *gz = malloc(sizeof(double) * F * N);
    double *gy = malloc(sizeof(double) * N);
    double *K = malloc(sizeof(double) * N), *Tx = malloc(sizeof(double) * n * (n + 1));
    double *Ty = malloc(sizeof(double) * n * (n + 1)), *u = malloc(sizeof(double) * N);
    memset(grad, 0, sizeof(double) * np);
    double L = 0.0;
    const double inv = 1.0 / ((double)B * (double)N);
    /* parameter offsets */
    const int64_t o_out = (int64_t)F * cin * 9 + F + (int64_t)R * (F * F * 9 + F);
    for (int s = 0; s < B; ++s) {
        oracle_cnn_forward(n, 1, cin, F, R, theta, x + (size_t)s * cin * N, y, z, h);
        if (kind == 0) {
            for (size_t k = 0; k < N; ++k) {
                const double d = y[k] - t[(size_t)s * N + k];
                L += d * d * inv;
                gy[k] = 2.0 * d * inv;
            }
        } else {
            /* u = x1 - A y; dL/dy = -2 A^T u / (B n^2), and A is symmetric */
            const double *x0 = x + (size_t)s * cin * N, *x1 = x0 + N;
            for (size_t k = 0; k < N; ++k) K[k] = exp(x0[k]);
            oracle_faces(n, K, 2, Tx, Ty);
            oracle_apply(n, Tx, Ty, y, u);
            for (size_t k = 0; k < N; ++k) {
                u[k] = x1[k] - u[k];
                L += u[k] * u[k] * inv;
            }
            oracle_apply(n, Tx, Ty, u, gy);
            for (size_t k = 0; k < N; ++k) gy[k] *= -2.0 * inv;
        }
        /* output layer */
        conv3_w(n, F, 1, gy, h + (size_t)R * F * N, grad + o_out, grad + o_out + F * 9);
        memset(gh, 0, sizeof(double) * F * N);
        conv3_t(n, F, 1, theta + o_out, gy, gh);
        /* residual layers, last to first: hk = h_{k-1} + relu(zk) */
        for (int l = R; l >= 1; --l) {
            const int64_t o = (int64_t)F * cin * 9 + F + (int64_t)(l - 1) * (F * F * 9 + F);
            const double *zl = z + (size_t)l * F * N;
            for (size_t k = 0; k < F * N; ++k) gz[k] = zl[k] > 0.0 ? gh[k] : 0.0;
            conv3_w(n, F, F, gz, h + (size_t)(l - 1) * F * N, grad + o, grad + o + F * F * 9);
            conv3_t(n, F, F, theta + o, gz, gh); /* gh becomes the gradient of h_{l-1} */
        }
        for (size_t k = 0; k < F * N; ++k) gz[k] = z[k] > 0.0 ? gh[k] : 0.0;
        conv3_w(n, cin, F, gz, x + (size_t)s * cin * N, grad, grad + F * cin * 9);
    }
    free(y);
    free(z);
    free(h);
    free(gh);
    free(gz);
    free(gy);
    free(K);
    free(Tx);
    free(Ty);
    free(u);
    return L;
}

double oracle_cnn_loss_grad(int n, int B, int cin, int F, int R, const double *theta, const double *x,
                            const double *t, double *grad)
{
    return oracle_cnn_loss_grad_kind(n, B, cin, F, R, theta, x, t, 0, grad);
}

/* One Adam step (step count t >= 1 after this update) on np parameters. */
void oracle_adam(int64_t np, double *theta, const double *g, double *m, double *v, int t, double lr,
                 double beta1, double beta2, double eps)
{
    const double c1 = 1.0 - pow(beta1, t), c2 = 1.0 - pow(beta2, t);
    for (int64_t k = 0; k < np; ++k) {
        m[k] = beta1 * m[k] + (1.0 - beta1) * g[k];
        v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k];
        const double mh = m[k] / c1, vh = v[k] / c2;
        theta[k] -= lr * mh / (sqrt(vh) + eps);
    }
}
