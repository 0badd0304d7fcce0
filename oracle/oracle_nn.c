/*
 * Serial FP64 CPU oracle of the learned preconditioner's network (a 3-level 3-D
 * convolutional U-Net) and its training step.  TEST INFRASTRUCTURE ONLY, like
 * oracle.c: nothing in the product library calls or links it, and it shares no code
 * with the HIP kernels.
 *
 * Tensors are channels-last: x[c * C + ch] for cell c = i + nr (j + nt k) of an
 * nr x nt x np grid (i radial, j polar, k azimuthal).  A 3x3x3 convolution has taps
 * t = (dk+1)*9 + (dj+1)*3 + (di+1); tap t of output cell (i, j, k) reads input cell
 * (i+di, j+dj, (k+dk) mod np), or zero when i+di or j+dj falls outside the grid
 * (zero padding in r and theta, periodic in phi).  Weights are w[(t * Cout + co) * Cin + ci].
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

static long nb_index(int nr, int nt, int np, int i, int j, int k, int t)
{
    int di = t % 3 - 1, dj = (t / 3) % 3 - 1, dk = t / 9 - 1;
    int a = i + di, b = j + dj, c = ((k + dk) % np + np) % np;
    if (a < 0 || a >= nr || b < 0 || b >= nt) return -1;
    return a + (long)nr * (b + (long)nt * c);
}

/* y = act(conv(x, w) + b); act = ReLU when relu != 0. */
void ognn_conv_fwd(int nr, int nt, int np, const double *x, int cin, const double *w, const double *b,
                   int cout, int relu, double *y)
{
    long n = (long)nr * nt * np;
    for (int k = 0; k < np; k++)
        for (int j = 0; j < nt; j++)
            for (int i = 0; i < nr; i++) {
                long c = i + (long)nr * (j + (long)nt * k);
                for (int co = 0; co < cout; co++) {
                    double s = b ? b[co] : 0.0;
                    for (int t = 0; t < 27; t++) {
                        long e = nb_index(nr, nt, np, i, j, k, t);
                        if (e < 0) continue;
                        for (int ci = 0; ci < cin; ci++) s += w[((long)t * cout + co) * cin + ci] * x[e * cin + ci];
                    }
                    y[c * cout + co] = (relu && s < 0.0) ? 0.0 : s;
                }
            }
    (void)n;
}

/* dx = d(conv)/dx^T dy: every (output cell, tap) that read input cell e sends
 * w * dy back to it (the adjoint of the gather above).  dx is overwritten. */
void ognn_conv_bwd_data(int nr, int nt, int np, const double *dy, int cout, const double *w, int cin, double *dx)
{
    long n = (long)nr * nt * np;
    memset(dx, 0, sizeof(double) * n * cin);
    for (int k = 0; k < np; k++)
        for (int j = 0; j < nt; j++)
            for (int i = 0; i < nr; i++) {
                long c = i + (long)nr * (j + (long)nt * k);
                for (int t = 0; t < 27; t++) {
                    long e = nb_index(nr, nt, np, i, j, k, t);
                    if (e < 0) continue;
                    for (int co = 0; co < cout; co++) {
                        double g = dy[c * cout + co];
                        for (int ci = 0; ci < cin; ci++) dx[e * cin + ci] += w[((long)t * cout + co) * cin + ci] * g;
                    }
                }
            }
}

/* dw[t][co][ci] = sum_c dy[c][co] x[nb(c, t)][ci];  db[co] = sum_c dy[c][co]. */
void ognn_conv_bwd_weight(int nr, int nt, int np, const double *x, int cin, const double *dy, int cout,
                          double *dw, double *db)
{
    memset(dw, 0, sizeof(double) * 27 * cout * cin);
    if (db) memset(db, 0, sizeof(double) * cout);
    for (int k = 0; k < np; k++)
        for (int j = 0; j < nt; j++)
            for (int i = 0; i < nr; i++) {
                long c = i + (long)nr * (j + (long)nt * k);
                for (int co = 0; co < cout; co++) {
                    double g = dy[c * cout + co];
                    if (db) db[co] += g;
                    for (int t = 0; t < 27; t++) {
                        long e = nb_index(nr, nt, np, i, j, k, t);
                        if (e < 0) continue;
                        for (int ci = 0; ci < cin; ci++) dw[((long)t * cout + co) * cin + ci] += g * x[e * cin + ci];
                    }
                }
            }
}

/* 2x2x2 average pooling of a (nr, nt, np) grid into (nr/2, nt/2, np/2). */
void ognn_pool(int nr, int nt, int np, const double *x, int C, double *y)
{
    int mr = nr / 2, mt = nt / 2, mp = np / 2;
    for (int K = 0; K < mp; K++)
        for (int J = 0; J < mt; J++)
            for (int I = 0; I < mr; I++)
                for (int ch = 0; ch < C; ch++) {
                    double s = 0.0;
                    for (int a = 0; a < 8; a++) {
                        long f = (2 * I + (a & 1)) + (long)nr * ((2 * J + ((a >> 1) & 1)) + (long)nt * (2 * K + (a >> 2)));
                        s += x[f * C + ch];
                    }
                    y[(I + (long)mr * (J + (long)mt * K)) * C + ch] = s / 8.0;
                }
}

/* Nearest-neighbour upsampling of a coarse (nr/2, nt/2, np/2) grid to (nr, nt, np). */
void ognn_up(int nr, int nt, int np, const double *xc, int C, double *y)
{
    int mr = nr / 2, mt = nt / 2;
    for (int k = 0; k < np; k++)
        for (int j = 0; j < nt; j++)
            for (int i = 0; i < nr; i++) {
                long f = i + (long)nr * (j + (long)nt * k), g = i / 2 + (long)mr * (j / 2 + (long)mt * (k / 2));
                for (int ch = 0; ch < C; ch++) y[f * C + ch] = xc[g * C + ch];
            }
}

/* ------------------------------------------------------------------ the U-Net
 *
 * Levels 0, 1, 2 at full, 1/2 and 1/4 resolution with 16, 32, 64 channels:
 *   L0: X(16) -> 16 relu        L1: 16 -> 16 relu  = S1
 *   pool -> L2: 16 -> 32 relu   L3: 32 -> 32 relu  = S2
 *   pool -> L4: 32 -> 64 relu   L5: 64 -> 64 relu  = B3
 *   L6: [up(B3) 64, S2 32] -> 32 relu   L7: 32 -> 32 relu = D2
 *   L8: [up(D2) 32, S1 16] -> 16 relu   L9: 16 -> 16 relu = D1
 *   L10: 1x1 conv 16 -> 1 (linear) = z
 * The input X has 16 channels (the residual, three operator features, zeros).
 */
#define NL 11
static const int CIN[NL] = {16, 16, 16, 32, 32, 64, 96, 32, 48, 16, 16};
static const int COUT[NL] = {16, 16, 32, 32, 64, 64, 32, 32, 16, 16, 1};
static const int LEVEL[NL] = {0, 0, 1, 1, 2, 2, 1, 1, 0, 0, 0};

int ognn_layers(void) { return NL; }
int ognn_cin(int l) { return CIN[l]; }
int ognn_cout(int l) { return COUT[l]; }
int ognn_taps(int l) { return l == NL - 1 ? 1 : 27; }

/* Offsets of layer l's weights and biases in one flat parameter vector:
 * [w0, b0, w1, b1, ...], w_l of size taps * Cout * Cin. */
long ognn_param_offset(int l)
{
    long o = 0;
    for (int m = 0; m < l; m++) o += (long)ognn_taps(m) * COUT[m] * CIN[m] + COUT[m];
    return o;
}
long ognn_param_count(void) { return ognn_param_offset(NL); }

static void dims(int nr, int nt, int np, int lev, int *r, int *t, int *p)
{
    *r = nr >> lev; *t = nt >> lev; *p = np >> lev;
}

/* Activations of one forward pass (allocated by ognn_forward, freed by ognn_free). */
typedef struct {
    double *a[NL];   /* outputs of layers 0..10 */
    double *p1, *p2; /* pooled S1, S2 */
    double *c6, *c8; /* concatenated inputs of layers 6 and 8 */
} ognn_acts;

void ognn_free(ognn_acts *A)
{
    for (int l = 0; l < NL; l++) free(A->a[l]);
    free(A->p1); free(A->p2); free(A->c6); free(A->c8);
    memset(A, 0, sizeof(*A));
}

static void concat(long n, const double *u, int cu, const double *s, int cs, double *out)
{
    for (long c = 0; c < n; c++) {
        memcpy(out + c * (cu + cs), u + c * cu, sizeof(double) * cu);
        memcpy(out + c * (cu + cs) + cu, s + c * cs, sizeof(double) * cs);
    }
}

/* 1x1 convolution 16 -> 1 (linear). */
static void conv1x1(long n, const double *x, int cin, const double *w, const double *b, double *z)
{
    for (long c = 0; c < n; c++) {
        double s = b[0];
        for (int ci = 0; ci < cin; ci++) s += w[ci] * x[c * cin + ci];
        z[c] = s;
    }
}

/* x rounded to the nearest bfloat16 (8 significant bits, ties to even), through the
 * nearest float; infinities and NaN pass unchanged.  Models the bf16 storage of the
 * network's activations (config: BF16 weights / activations, FP32 accumulation). */
static double bf16_round(double x)
{
    float f = (float)x;
    unsigned u;
    memcpy(&u, &f, sizeof u);
    if ((u & 0x7f800000u) == 0x7f800000u) return f;
    u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
    memcpy(&f, &u, sizeof f);
    return f;
}

static void round_all(long n, double *x, int quant)
{
    if (!quant) return;
    for (long i = 0; i < n; i++) x[i] = bf16_round(x[i]);
}

double ognn_bf16_round(double x) { return bf16_round(x); }

/* Forward pass: X [n0][16] -> z [n0]; keeps every activation in *A.  quant != 0 stores
 * every layer output (after the ReLU) and every pooled tensor as bf16, as the matrix-core
 * kernels do; the 1x1 output layer stays unrounded. */
static void forward_impl(int nr, int nt, int np, const double *params, const double *X, ognn_acts *A, double *z,
                         int quant)
{
    int r[3], t[3], p[3];
    long n[3];
    for (int lev = 0; lev < 3; lev++) {
        dims(nr, nt, np, lev, &r[lev], &t[lev], &p[lev]);
        n[lev] = (long)r[lev] * t[lev] * p[lev];
    }
    memset(A, 0, sizeof(*A));
    for (int l = 0; l < NL - 1; l++) A->a[l] = (double *)malloc(sizeof(double) * n[LEVEL[l]] * COUT[l]);
    A->a[NL - 1] = (double *)malloc(sizeof(double) * n[0]);
    A->p1 = (double *)malloc(sizeof(double) * n[1] * 16);
    A->p2 = (double *)malloc(sizeof(double) * n[2] * 32);
    A->c6 = (double *)malloc(sizeof(double) * n[1] * 96);
    A->c8 = (double *)malloc(sizeof(double) * n[0] * 48);
    double *up6 = (double *)malloc(sizeof(double) * n[1] * 64), *up8 = (double *)malloc(sizeof(double) * n[0] * 32);
#define W(l) (params + ognn_param_offset(l))
#define B(l) (params + ognn_param_offset(l) + (long)ognn_taps(l) * COUT[l] * CIN[l])
    ognn_conv_fwd(r[0], t[0], p[0], X, 16, W(0), B(0), 16, 1, A->a[0]);
    round_all(n[0] * 16, A->a[0], quant);
    ognn_conv_fwd(r[0], t[0], p[0], A->a[0], 16, W(1), B(1), 16, 1, A->a[1]);
    round_all(n[0] * 16, A->a[1], quant);
    ognn_pool(r[0], t[0], p[0], A->a[1], 16, A->p1);
    round_all(n[1] * 16, A->p1, quant);
    ognn_conv_fwd(r[1], t[1], p[1], A->p1, 16, W(2), B(2), 32, 1, A->a[2]);
    round_all(n[1] * 32, A->a[2], quant);
    ognn_conv_fwd(r[1], t[1], p[1], A->a[2], 32, W(3), B(3), 32, 1, A->a[3]);
    round_all(n[1] * 32, A->a[3], quant);
    ognn_pool(r[1], t[1], p[1], A->a[3], 32, A->p2);
    round_all(n[2] * 32, A->p2, quant);
    ognn_conv_fwd(r[2], t[2], p[2], A->p2, 32, W(4), B(4), 64, 1, A->a[4]);
    round_all(n[2] * 64, A->a[4], quant);
    ognn_conv_fwd(r[2], t[2], p[2], A->a[4], 64, W(5), B(5), 64, 1, A->a[5]);
    round_all(n[2] * 64, A->a[5], quant);
    ognn_up(r[1], t[1], p[1], A->a[5], 64, up6);
    concat(n[1], up6, 64, A->a[3], 32, A->c6);
    ognn_conv_fwd(r[1], t[1], p[1], A->c6, 96, W(6), B(6), 32, 1, A->a[6]);
    round_all(n[1] * 32, A->a[6], quant);
    ognn_conv_fwd(r[1], t[1], p[1], A->a[6], 32, W(7), B(7), 32, 1, A->a[7]);
    round_all(n[1] * 32, A->a[7], quant);
    ognn_up(r[0], t[0], p[0], A->a[7], 32, up8);
    concat(n[0], up8, 32, A->a[1], 16, A->c8);
    ognn_conv_fwd(r[0], t[0], p[0], A->c8, 48, W(8), B(8), 16, 1, A->a[8]);
    round_all(n[0] * 16, A->a[8], quant);
    ognn_conv_fwd(r[0], t[0], p[0], A->a[8], 16, W(9), B(9), 16, 1, A->a[9]);
    round_all(n[0] * 16, A->a[9], quant);
    conv1x1(n[0], A->a[9], 16, W(10), B(10), A->a[10]);
    memcpy(z, A->a[10], sizeof(double) * n[0]);
    free(up6); free(up8);
}

void ognn_forward(int nr, int nt, int np, const double *params, const double *X, ognn_acts *A, double *z)
{
    forward_impl(nr, nt, np, params, X, A, z, 0);
}

/* The forward pass with bf16 activations (forward_impl with quant = 1): z [n0]. */
void ognn_forward_bf16(int nr, int nt, int np, const double *params, const double *X, double *z)
{
    ognn_acts A;
    forward_impl(nr, nt, np, params, X, &A, z, 1);
    ognn_free(&A);
}

/* dx *= (y > 0): ReLU backward from the layer output. */
static void relu_bwd(long n, const double *y, double *g)
{
    for (long c = 0; c < n; c++)
        if (!(y[c] > 0.0)) g[c] = 0.0;
}

static void pool_bwd(int nr, int nt, int np, const double *dyc, int C, double *dx_add)
{
    int mr = nr / 2, mt = nt / 2;
    for (int k = 0; k < np; k++)
        for (int j = 0; j < nt; j++)
            for (int i = 0; i < nr; i++) {
                long f = i + (long)nr * (j + (long)nt * k), g = i / 2 + (long)mr * (j / 2 + (long)mt * (k / 2));
                for (int ch = 0; ch < C; ch++) dx_add[f * C + ch] += dyc[g * C + ch] / 8.0;
            }
}

static void up_bwd(int nr, int nt, int np, const double *dyf, int Cf, int c0, int C, double *dxc)
{
    int mr = nr / 2, mt = nt / 2;
    memset(dxc, 0, sizeof(double) * (long)mr * mt * (np / 2) * C);
    for (int k = 0; k < np; k++)
        for (int j = 0; j < nt; j++)
            for (int i = 0; i < nr; i++) {
                long f = i + (long)nr * (j + (long)nt * k), g = i / 2 + (long)mr * (j / 2 + (long)mt * (k / 2));
                for (int ch = 0; ch < C; ch++) dxc[g * C + ch] += dyf[f * Cf + c0 + ch];
            }
}

/* Backward pass for dL/dz = gz: gradients of all parameters into grad (same layout
 * as params).  Also returns dL/dX in gX if not NULL. */
void ognn_backward(int nr, int nt, int np, const double *params, const double *X, const ognn_acts *A,
                   const double *gz, double *grad, double *gX)
{
    int r[3], t[3], p[3];
    long n[3];
    for (int lev = 0; lev < 3; lev++) {
        dims(nr, nt, np, lev, &r[lev], &t[lev], &p[lev]);
        n[lev] = (long)r[lev] * t[lev] * p[lev];
    }
#define GW(l) (grad + ognn_param_offset(l))
#define GB(l) (grad + ognn_param_offset(l) + (long)ognn_taps(l) * COUT[l] * CIN[l])
    double *g9 = (double *)calloc(n[0] * 16, sizeof(double));
    /* layer 10 (1x1) */
    memset(GW(10), 0, sizeof(double) * 17);
    for (long c = 0; c < n[0]; c++) {
        GB(10)[0] += gz[c];
        for (int ci = 0; ci < 16; ci++) {
            GW(10)[ci] += gz[c] * A->a[9][c * 16 + ci];
            g9[c * 16 + ci] = W(10)[ci] * gz[c];
        }
    }
    /* layer 9 */
    relu_bwd(n[0] * 16, A->a[9], g9);
    double *g8 = (double *)malloc(sizeof(double) * n[0] * 16);
    ognn_conv_bwd_weight(r[0], t[0], p[0], A->a[8], 16, g9, 16, GW(9), GB(9));
    ognn_conv_bwd_data(r[0], t[0], p[0], g9, 16, W(9), 16, g8);
    /* layer 8: input c8 = [up(a7) 32, a1 16] */
    relu_bwd(n[0] * 16, A->a[8], g8);
    double *gc8 = (double *)malloc(sizeof(double) * n[0] * 48);
    ognn_conv_bwd_weight(r[0], t[0], p[0], A->c8, 48, g8, 16, GW(8), GB(8));
    ognn_conv_bwd_data(r[0], t[0], p[0], g8, 16, W(8), 48, gc8);
    double *g7 = (double *)malloc(sizeof(double) * n[1] * 32);
    up_bwd(r[0], t[0], p[0], gc8, 48, 0, 32, g7);
    double *g1 = (double *)malloc(sizeof(double) * n[0] * 16);
    for (long c = 0; c < n[0]; c++)
        for (int ch = 0; ch < 16; ch++) g1[c * 16 + ch] = gc8[c * 48 + 32 + ch];
    /* layer 7 */
    relu_bwd(n[1] * 32, A->a[7], g7);
    double *g6 = (double *)malloc(sizeof(double) * n[1] * 32);
    ognn_conv_bwd_weight(r[1], t[1], p[1], A->a[6], 32, g7, 32, GW(7), GB(7));
    ognn_conv_bwd_data(r[1], t[1], p[1], g7, 32, W(7), 32, g6);
    /* layer 6: input c6 = [up(a5) 64, a3 32] */
    relu_bwd(n[1] * 32, A->a[6], g6);
    double *gc6 = (double *)malloc(sizeof(double) * n[1] * 96);
    ognn_conv_bwd_weight(r[1], t[1], p[1], A->c6, 96, g6, 32, GW(6), GB(6));
    ognn_conv_bwd_data(r[1], t[1], p[1], g6, 32, W(6), 96, gc6);
    double *g5 = (double *)malloc(sizeof(double) * n[2] * 64);
    up_bwd(r[1], t[1], p[1], gc6, 96, 0, 64, g5);
    double *g3 = (double *)malloc(sizeof(double) * n[1] * 32);
    for (long c = 0; c < n[1]; c++)
        for (int ch = 0; ch < 32; ch++) g3[c * 32 + ch] = gc6[c * 96 + 64 + ch];
    /* layer 5, 4 */
    relu_bwd(n[2] * 64, A->a[5], g5);
    double *g4 = (double *)malloc(sizeof(double) * n[2] * 64);
    ognn_conv_bwd_weight(r[2], t[2], p[2], A->a[4], 64, g5, 64, GW(5), GB(5));
    ognn_conv_bwd_data(r[2], t[2], p[2], g5, 64, W(5), 64, g4);
    relu_bwd(n[2] * 64, A->a[4], g4);
    double *gp2 = (double *)malloc(sizeof(double) * n[2] * 32);
    ognn_conv_bwd_weight(r[2], t[2], p[2], A->p2, 32, g4, 64, GW(4), GB(4));
    ognn_conv_bwd_data(r[2], t[2], p[2], g4, 64, W(4), 32, gp2);
    pool_bwd(r[1], t[1], p[1], gp2, 32, g3);
    /* layer 3, 2 */
    relu_bwd(n[1] * 32, A->a[3], g3);
    double *g2 = (double *)malloc(sizeof(double) * n[1] * 32);
    ognn_conv_bwd_weight(r[1], t[1], p[1], A->a[2], 32, g3, 32, GW(3), GB(3));
    ognn_conv_bwd_data(r[1], t[1], p[1], g3, 32, W(3), 32, g2);
    relu_bwd(n[1] * 32, A->a[2], g2);
    double *gp1 = (double *)malloc(sizeof(double) * n[1] * 16);
    ognn_conv_bwd_weight(r[1], t[1], p[1], A->p1, 16, g2, 32, GW(2), GB(2));
    ognn_conv_bwd_data(r[1], t[1], p[1], g2, 32, W(2), 16, gp1);
    pool_bwd(r[0], t[0], p[0], gp1, 16, g1);
    /* layer 1, 0 */
    relu_bwd(n[0] * 16, A->a[1], g1);
    double *g0 = (double *)malloc(sizeof(double) * n[0] * 16);
    ognn_conv_bwd_weight(r[0], t[0], p[0], A->a[0], 16, g1, 16, GW(1), GB(1));
    ognn_conv_bwd_data(r[0], t[0], p[0], g1, 16, W(1), 16, g0);
    relu_bwd(n[0] * 16, A->a[0], g0);
    ognn_conv_bwd_weight(r[0], t[0], p[0], X, 16, g0, 16, GW(0), GB(0));
    if (gX) ognn_conv_bwd_data(r[0], t[0], p[0], g0, 16, W(0), 16, gX);
    free(g9); free(g8); free(gc8); free(g7); free(g1); free(g6); free(gc6); free(g5); free(g3);
    free(g4); free(gp2); free(g2); free(gp1); free(g0);
}

/* Loss L = ||z - e||^2 / ||e||^2 and dL/dz. */
double ognn_loss(long n, const double *z, const double *e, double *gz)
{
    double num = 0.0, den = 0.0;
    for (long c = 0; c < n; c++) {
        double d = z[c] - e[c];
        num += d * d;
        den += e[c] * e[c];
    }
    if (gz)
        for (long c = 0; c < n; c++) gz[c] = 2.0 * (z[c] - e[c]) / den;
    return num / den;
}

/* One Adam step (Kingma & Ba) with bias correction, step index t >= 1. */
void ognn_adam(long n, double *p, const double *g, double *m, double *v, double lr, double b1, double b2,
               double eps, int t)
{
    double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (long i = 0; i < n; i++) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        p[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* Convenience: forward + loss + backward in one call (returns the loss). */
double ognn_loss_grad(int nr, int nt, int np, const double *params, const double *X, const double *e,
                      double *grad, double *z)
{
    long n = (long)nr * nt * np;
    ognn_acts A;
    double *zz = z ? z : (double *)malloc(sizeof(double) * n);
    double *gz = (double *)malloc(sizeof(double) * n);
    ognn_forward(nr, nt, np, params, X, &A, zz);
    double L = ognn_loss(n, zz, e, gz);
    ognn_backward(nr, nt, np, params, X, &A, gz, grad, NULL);
    ognn_free(&A);
    free(gz);
    if (!z) free(zz);
    return L;
}

/* q = A z for the Jacobi-scaled operator: unit diagonal, ahat[c], ahat[n + c] and
 * ahat[2n + c] the coefficients between cell c and its outward radial, polar and
 * azimuthal (periodic) neighbours. */
static void scaled_apply(int nr, int nt, int np, const double *ahat, const double *z, double *q)
{
    long n = (long)nr * nt * np;
    const double *ar = ahat, *at = ahat + n, *ap = ahat + 2 * n;
    for (int k = 0; k < np; k++)
        for (int j = 0; j < nt; j++)
            for (int i = 0; i < nr; i++) {
                long c = i + (long)nr * (j + (long)nt * k);
                double v = z[c];
                if (i + 1 < nr) v += ar[c] * z[c + 1];
                if (i > 0) v += ar[c - 1] * z[c - 1];
                if (j + 1 < nt) v += at[c] * z[c + nr];
                if (j > 0) v += at[c - nr] * z[c - nr];
                if (np > 1) {
                    long kp = i + (long)nr * (j + (long)nt * ((k + 1) % np));
                    long km = i + (long)nr * (j + (long)nt * ((k + np - 1) % np));
                    v += ap[c] * z[kp] + ap[km] * z[km];
                }
                q[c] = v;
            }
}

/* Residual loss of the network as a preconditioner: L = ||A z - r||^2 / ||r||^2 with
 * z = U-Net(X), and its parameter gradient: dL/d(Az) = 2 (A z - r) / ||r||^2, then
 * dL/dz = A dL/d(Az) (A symmetric), then the backward pass. */
double ognn_loss_grad_resid(int nr, int nt, int np, const double *params, const double *X, const double *r,
                            const double *ahat, double *grad, double *z)
{
    long n = (long)nr * nt * np;
    ognn_acts A;
    double *zz = z ? z : (double *)malloc(sizeof(double) * n);
    double *q = (double *)malloc(sizeof(double) * n);
    double *gq = (double *)malloc(sizeof(double) * n);
    double *gz = (double *)malloc(sizeof(double) * n);
    ognn_forward(nr, nt, np, params, X, &A, zz);
    scaled_apply(nr, nt, np, ahat, zz, q);
    double L = ognn_loss(n, q, r, gq);
    scaled_apply(nr, nt, np, ahat, gq, gz);
    ognn_backward(nr, nt, np, params, X, &A, gz, grad, NULL);
    ognn_free(&A);
    free(q);
    free(gq);
    free(gz);
    if (!z) free(zz);
    return L;
}
