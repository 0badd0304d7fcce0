/*
 * Serial FP64 CPU oracle of the radiation step of Kuiper et al., "Fast and accurate
 * frequency dependent radiation transport for hydrodynamics simulations in massive
 * star formation".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may call, link or load
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no source with the HIP path: constants, geometry,
 * table lookups and solvers are written out again here, in the paper's order, for a
 * reader to check against the paper by eye.  Nothing is blocked, fused or reordered.
 *
 * The same source also builds with OpenMP (-fopenmp; the CPU baseline on all host
 * cores, and the oracle side of the tests on the largest grids): the loops over
 * radial columns and cells are split over threads, each cell computed exactly as in
 * the serial build.  Only the sums over all cells (dot products, norms) change order
 * there: fixed 4096-cell blocks summed in parallel, then the block sums in block order,
 * so the result does not depend on the thread count.
 *
 * Layout: cell (i, j, k) of an N_r x N_theta x N_phi spherical-polar grid has index
 * c = i + N_r (j + N_theta k) (r fastest).  Radial face i (at r_face[i], i = 0..N_r)
 * of column (j, k) has index i + (N_r + 1)(j + N_theta k).
 *
 * Readings of points the paper leaves open (each one flagged again where it is used):
 *  R1  Eq. (20): the bin flux is pi * int B_nu dnu over the bin (the c/4 of the
 *      printed equation multiplies the energy density 4 pi B_nu / c); the first bin
 *      starts at nu = 0 and the last ends at infinity.
 *  R2  Per-bin opacity: kappa at the bin mid-frequency (Sect. "Frequency dependent
 *      irradiation").  Table lookup: kappa_nu linear in T between nodes, kappa_P and
 *      kappa_R linear in log-log; clamped to the end nodes outside the table.
 *  R3  |F_*|/c at a cell in Eq. (16) (fluxes live on faces): the cell-integrated
 *      absorbed flux, kappa_nu Fbar_nu = q_nu / rho, as in Eqs. (28)-(32).
 *  R4  FLD faces (not given): (kappa_R rho) and E at a face are arithmetic means of
 *      the two cells; R uses the normal difference only; coefficients are lagged at
 *      (E^n, T^n).  For R > 1e100 the limiter is taken as its limit 1/R.
 *  R5  Outer radial boundary: one ghost cell continuing the radial stretching, with
 *      rho_ghost = rho_last, kappa_R at T_bc and E_ghost = a T_bc^4 (Dirichlet);
 *      inner radial face and both poles carry zero flux; phi is periodic.
 *  R6  Time discretisation: backward Euler, one linear solve per step.
 *  R7  Relative residual: ||b^ - A^ y||_2 / ||b^||_2 of the Jacobi-scaled symmetric
 *      system, starting from y = E^n / s.
 *  R8  Newton on Eq. (16): g(T) = a T^4 - E - S/kappa_P(T), started at T^n, kept in
 *      a bracket that isolates the smallest root (bisection when a step leaves it),
 *      stopped when the Newton step is <= 1e-14 T or after 50 iterations.
 *  R9  Thermal force at a cell: mean of the two face fluxes per direction times
 *      kappa_R rho / c (Eq. (27) with the FLD flux of Eq. (10)).
 *  R20 Runs without diffusion (the pure-absorption rows of the run table): the thermal
 *      radiation field is never transported and stays at the background a T_bc^4, so
 *      Eq. (16) balances the absorbed stellar power against re-emission cell by cell.
 *      Gray irradiation (Eqs. (18)-(19)) is the one-bin case with the total flux
 *      sigma T_*^4 = sum_b F_b and, at each table temperature, the F_b-weighted mean of
 *      the bin opacities (the Planck mean at T_*, keeping the table's dust-temperature
 *      dependence).  The main iteration stops when the largest relative temperature
 *      change of a step is below the threshold (0.01 % in the run setup).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* CGS constants (CODATA 2018). */
#define OG_C 2.99792458e10
#define OG_H 6.62607015e-27
#define OG_KB 1.380649e-16
#define OG_SIGMA 5.670374419e-5
#define OG_A (4.0 * OG_SIGMA / OG_C) /* radiation constant; sigma = a c / 4 (Eq. 18) */
#define OG_PI 3.14159265358979323846

typedef struct {
    int nr, nt, np;
    const double *rf, *tf, *pf; /* faces: nr+1, nt+1, np+1 */
} og_grid;

typedef struct {
    int nT, nnu;
    const double *T;    /* nT nodes, increasing */
    const double *kap;  /* nT x nnu, row-major */
    const double *kapP; /* nT */
    const double *kapR; /* nT */
} og_opac;

typedef struct {
    double R, Teff;
    const double *F0; /* nnu bin fluxes at the stellar surface */
} og_star;

typedef struct {
    double dt, cV, Tbc, Efloor;
} og_fld;

double og_const_a(void) { return OG_A; }
double og_const_c(void) { return OG_C; }

/* ------------------------------------------------------------------ geometry */

static double rc(const og_grid *g, int i) { return 0.5 * (g->rf[i] + g->rf[i + 1]); }
static double tc(const og_grid *g, int j) { return 0.5 * (g->tf[j] + g->tf[j + 1]); }
static double pc(const og_grid *g, int k) { return 0.5 * (g->pf[k] + g->pf[k + 1]); }
static double dphi(const og_grid *g, int k) { return g->pf[k + 1] - g->pf[k]; }
static double dcos(const og_grid *g, int j) { return cos(g->tf[j]) - cos(g->tf[j + 1]); }

static double volume(const og_grid *g, int i, int j, int k)
{
    double r0 = g->rf[i], r1 = g->rf[i + 1];
    return (r1 * r1 * r1 - r0 * r0 * r0) / 3.0 * dcos(g, j) * dphi(g, k);
}

/* Area of the radial face at r_face[i] within column (j, k). */
static double area_r(const og_grid *g, int i, int j, int k)
{
    double r = g->rf[i];
    return r * r * dcos(g, j) * dphi(g, k);
}

/* Area of the polar face at th_face[j] within (i, k). */
static double area_t(const og_grid *g, int i, int j, int k)
{
    double r0 = g->rf[i], r1 = g->rf[i + 1];
    return sin(g->tf[j]) * 0.5 * (r1 * r1 - r0 * r0) * dphi(g, k);
}

/* Area of the azimuthal face at ph_face[k] within (i, j) (independent of k). */
static double area_p(const og_grid *g, int i, int j)
{
    double r0 = g->rf[i], r1 = g->rf[i + 1];
    return 0.5 * (r1 * r1 - r0 * r0) * (g->tf[j + 1] - g->tf[j]);
}

/* Centre of the outer ghost cell (R5): the last cell's stretching continued once. */
static double rc_ghost(const og_grid *g)
{
    double rlast = g->rf[g->nr], rprev = g->rf[g->nr - 1];
    double rg = rlast * (rlast / rprev);
    return 0.5 * (rlast + rg);
}

/* Centre-to-centre distances across the outward faces of cell (i, j, k). */
static double ds_r(const og_grid *g, int i)
{
    return (i + 1 < g->nr) ? rc(g, i + 1) - rc(g, i) : rc_ghost(g) - rc(g, i);
}
static double ds_t(const og_grid *g, int i, int j) { return rc(g, i) * (tc(g, j + 1) - tc(g, j)); }
static double ds_p(const og_grid *g, int i, int j, int k)
{
    double d;
    if (k + 1 < g->np)
        d = pc(g, k + 1) - pc(g, k);
    else /* periodic wrap */
        d = (g->pf[g->np] - pc(g, k)) + (pc(g, 0) - g->pf[0]);
    return rc(g, i) * sin(tc(g, j)) * d;
}

static long cidx(const og_grid *g, int i, int j, int k) { return i + (long)g->nr * (j + (long)g->nt * k); }
static long fidx(const og_grid *g, int i, int j, int k) { return i + (long)(g->nr + 1) * (j + (long)g->nt * k); }

/* ------------------------------------------------------------- opacity (R2) */

/* Node k and linear weight w with T_k <= T <= T_{k+1}, clamped to the table. */
static void lookup(const og_opac *op, double T, int *kk, double *w)
{
    int n = op->nT;
    if (T <= op->T[0]) { *kk = 0; *w = 0.0; return; }
    if (T >= op->T[n - 1]) { *kk = n - 2; *w = 1.0; return; }
    int k = 0;
    while (op->T[k + 1] <= T) k++;
    *kk = k;
    *w = (T - op->T[k]) / (op->T[k + 1] - op->T[k]);
}

double og_kappa_nu(const og_opac *op, double T, int b)
{
    int k; double w;
    lookup(op, T, &k, &w);
    return (1.0 - w) * op->kap[(long)k * op->nnu + b] + w * op->kap[(long)(k + 1) * op->nnu + b];
}

/* log-log interpolation of a mean-opacity column; *slope = d ln kappa / d ln T. */
static double loglog(const og_opac *op, const double *tab, double T, double *slope)
{
    int n = op->nT;
    if (T <= op->T[0]) { if (slope) *slope = 0.0; return tab[0]; }
    if (T >= op->T[n - 1]) { if (slope) *slope = 0.0; return tab[n - 1]; }
    int k = 0;
    while (op->T[k + 1] <= T) k++;
    double l0 = log(op->T[k]), l1 = log(op->T[k + 1]);
    double y0 = log(tab[k]), y1 = log(tab[k + 1]);
    double lw = (log(T) - l0) / (l1 - l0);
    if (slope) *slope = (y1 - y0) / (l1 - l0);
    return exp((1.0 - lw) * y0 + lw * y1);
}

double og_kappa_P(const og_opac *op, double T) { return loglog(op, op->kapP, T, NULL); }
double og_kappa_R(const og_opac *op, double T) { return loglog(op, op->kapR, T, NULL); }

/* -------------------------------------------------- stellar bin flux, Eq. (20) */

/* Planck integrand in x = h nu / (k T): x^3 / (e^x - 1). */
static double planck_x(double x) { return x > 0.0 ? x * x * x / expm1(x) : 0.0; }

/* n-point Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n. */
static void gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < (n + 1) / 2; i++) {
        double z = cos(OG_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = 0.0;
            for (int m = 1; m <= n; m++) {
                double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p2) / m;
            }
            dp = n * (z * p0 - p1) / (z * z - 1.0);
            double dz = p0 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        x[i] = -z; x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* int_a^b planck_x by composite 16-point Gauss-Legendre on panels of width <= 0.25. */
static double planck_integral(double a, double b)
{
    double gx[16], gw[16];
    gauss_legendre(16, gx, gw);
    int npan = (int)ceil((b - a) / 0.25);
    if (npan < 1) npan = 1;
    double h = (b - a) / npan, sum = 0.0;
    for (int p = 0; p < npan; p++) {
        double lo = a + p * h, mid = lo + 0.5 * h, part = 0.0;
        for (int m = 0; m < 16; m++) part += gw[m] * planck_x(mid + 0.5 * h * gx[m]);
        sum += 0.5 * h * part;
    }
    return sum;
}

/* Eq. (20) with reading R1: F_i = pi int_{bin i} B_nu(T_*) dnu
 *   = sigma T^4 (15/pi^4) int_{x_lo}^{x_hi} x^3/(e^x-1) dx,
 * bin edges at the midpoints between neighbouring mid-frequencies, 0 and infinity
 * at the ends (the integrand is below 1e-300 beyond x = 800). */
int og_star_bins(double Teff, int nnu, const double *nu, double *F0)
{
    if (nnu < 1 || Teff <= 0) return -1;
    double xs = OG_H / (OG_KB * Teff);
    double norm = OG_SIGMA * pow(Teff, 4) * 15.0 / pow(OG_PI, 4);
    for (int i = 0; i < nnu; i++) {
        double lo = (i == 0) ? 0.0 : 0.5 * (nu[i - 1] + nu[i]) * xs;
        double hi = (i == nnu - 1) ? 800.0 : 0.5 * (nu[i] + nu[i + 1]) * xs;
        if (lo > 800.0) lo = 800.0;
        if (hi > 800.0) hi = 800.0;
        F0[i] = hi > lo ? norm * planck_integral(lo, hi) : 0.0;
    }
    return 0;
}

/* -------------------------------------------------- ray trace, Eqs. (17)-(20) */

/* phi(x) = (1 - e^-x)/x, phi(0) = 1. */
static double phi1(double x) { return x == 0.0 ? 1.0 : -expm1(-x) / x; }

/*
 * Frequency-dependent first-order ray trace along the radial rays (Sect.
 * "Irradiation", Eqs. 17 and 19, and "Frequency dependent irradiation", Eq. 20).
 * Per column and bin: tau(r_in) = 0 (optically empty inner hole), tau grows by
 * kappa_nu(T_i) rho_i dr_i through cell i (Eq. 19 with kappa(nu) in place of
 * kappa_P(T_*)), F_nu(r) = F_nu(R_*) (R_* / r)^2 exp(-tau) at each face (Eq. 17).
 * Outputs, summed over bins in ascending order:
 *   q     - absorbed stellar power per volume, the spherical form of Eqs. (28)-(33)
 *           and (36): q = (A_- F_- - A_+ F_+)/V = 3 R_*^2 F_nu(R_*) e^{-tau_-}
 *           (1 - e^{-dtau}) / (r_+^3 - r_-^3);
 *   S     - sum_nu kappa_nu Fbar_nu / c = q_nu / (rho c) (reading R3), written with
 *           phi(dtau) so that it stays finite as rho -> 0;
 *   Fface - total stellar flux at every radial face (may be NULL);
 *   Fnu   - the flux of every bin at every radial face, F_nu(R_star) (R_star / r)^2 e^-tau_nu,
 *           bin fastest: Fnu[face index * n_nu + bin] (may be NULL).
 */
void og_raytrace(const og_grid *g, const og_opac *op, const og_star *st,
                 const double *rho, const double *T, double *q, double *S, double *Fface,
                 double *Fnu)
{
    int nr = g->nr, nt = g->nt, np = g->np, nnu = op->nnu;
    double R2 = st->R * st->R;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < np; k++)
        for (int j = 0; j < nt; j++) {
            for (int i = 0; i < nr; i++) {
                q[cidx(g, i, j, k)] = 0.0;
                S[cidx(g, i, j, k)] = 0.0;
            }
            if (Fface)
                for (int i = 0; i <= nr; i++) Fface[fidx(g, i, j, k)] = 0.0;
            for (int b = 0; b < nnu; b++) {
                double tau = 0.0;
                if (Fface) Fface[fidx(g, 0, j, k)] += st->F0[b] * R2 / (g->rf[0] * g->rf[0]);
                if (Fnu) Fnu[fidx(g, 0, j, k) * nnu + b] = st->F0[b] * R2 / (g->rf[0] * g->rf[0]);
                for (int i = 0; i < nr; i++) {
                    long c = cidx(g, i, j, k);
                    double r0 = g->rf[i], r1 = g->rf[i + 1], dr = r1 - r0;
                    double kap = og_kappa_nu(op, T[c], b);
                    double dtau = kap * rho[c] * dr;
                    double tau_in = tau;
                    tau = tau + dtau;
                    double G = 3.0 * R2 * st->F0[b] * exp(-tau_in) / (r1 * r1 * r1 - r0 * r0 * r0);
                    q[c] += G * (-expm1(-dtau));
                    S[c] += G * kap * dr * phi1(dtau) / OG_C;
                    if (Fface) Fface[fidx(g, i + 1, j, k)] += st->F0[b] * R2 / (r1 * r1) * exp(-tau);
                    if (Fnu) Fnu[fidx(g, i + 1, j, k) * nnu + b] = st->F0[b] * R2 / (r1 * r1) * exp(-tau);
                }
            }
        }
}

/* ------------------------------------------- radiation energy from T, Eq. (16) */

/* Fig. 1 "Radiation Energy": E^n = a T^4 - S / kappa_P(T) (Eq. 16 solved for E),
 * floored at Efloor. */
void og_energy(const og_grid *g, const og_opac *op, const og_fld *f,
               const double *T, const double *S, double *E)
{
    long n = (long)g->nr * g->nt * g->np;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; c++) {
        double t = T[c];
        double e = OG_A * t * t * t * t - S[c] / og_kappa_P(op, t);
        E[c] = e > f->Efloor ? e : f->Efloor;
    }
}

/* ---------------------------------------------- FLD assembly, Eqs. (8)-(15) */

/* Diffusion coefficient at a face (Eqs. 11-13 with reading R4). */
static double face_D(double chi_a, double chi_b, double Ea, double Eb, double ds)
{
    double chi = 0.5 * (chi_a + chi_b);
    double Ef = 0.5 * (Ea + Eb);
    double R = fabs(Eb - Ea) / (ds * chi * Ef);              /* Eq. 13 */
    double lam = R < 1e100 ? (2.0 + R) / (6.0 + 3.0 * R + R * R) : 1.0 / R; /* Eq. 12 */
    return OG_C * lam / chi;                                  /* Eq. 11 */
}

/*
 * Backward-Euler discretisation of Eq. (15) in finite-volume form (R6):
 *   V/(dt f_c) (E - E^n) = sum_faces w_f (E_nb - E) + V (q + Q+),
 *   f_c = (c_V rho / (4 a T^3) + 1)^-1 (Eq. 9),  w_f = A_f D_f / ds_f.
 * Writes the unscaled outward weights w[3n] (components r, theta, phi; the radial
 * weight of the last cell is the Dirichlet face of R5, theta weight of the last polar
 * cell is 0, phi weight 0 when N_phi = 1), the diagonal d, rhs b, the Jacobi scale
 * s = d^-1/2, the scaled off-diagonals ahat[3n] = -w s_c s_nb (0 on boundary faces)
 * and bhat = s b.  Q may be NULL.
 */
void og_assemble(const og_grid *g, const og_opac *op, const og_fld *f,
                 const double *rho, const double *T, const double *En, const double *q,
                 const double *Q, double *w, double *d, double *b, double *s,
                 double *ahat, double *bhat)
{
    int nr = g->nr, nt = g->nt, np = g->np;
    long n = (long)nr * nt * np;
    double *chi = (double *)malloc(sizeof(double) * n);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; c++) chi[c] = og_kappa_R(op, T[c]) * rho[c];
    double Eb = OG_A * pow(f->Tbc, 4);
    double *wr = w, *wt = w + n, *wp = w + 2 * n;

    /* outward face weights */
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < np; k++)
        for (int j = 0; j < nt; j++)
            for (int i = 0; i < nr; i++) {
                long c = cidx(g, i, j, k);
                if (i + 1 < nr) {
                    long e = cidx(g, i + 1, j, k);
                    double ds = ds_r(g, i);
                    wr[c] = area_r(g, i + 1, j, k) * face_D(chi[c], chi[e], En[c], En[e], ds) / ds;
                } else { /* Dirichlet ghost (R5) */
                    double chig = og_kappa_R(op, f->Tbc) * rho[c];
                    double ds = ds_r(g, i);
                    wr[c] = area_r(g, nr, j, k) * face_D(chi[c], chig, En[c], Eb, ds) / ds;
                }
                if (j + 1 < nt) {
                    long e = cidx(g, i, j + 1, k);
                    double ds = ds_t(g, i, j);
                    wt[c] = area_t(g, i, j + 1, k) * face_D(chi[c], chi[e], En[c], En[e], ds) / ds;
                } else
                    wt[c] = 0.0; /* pole: zero flux */
                if (np > 1) {
                    long e = cidx(g, i, j, (k + 1) % np);
                    double ds = ds_p(g, i, j, k);
                    wp[c] = area_p(g, i, j) * face_D(chi[c], chi[e], En[c], En[e], ds) / ds;
                } else
                    wp[c] = 0.0;
            }

    /* diagonal, rhs, Jacobi scale */
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < np; k++)
        for (int j = 0; j < nt; j++)
            for (int i = 0; i < nr; i++) {
                long c = cidx(g, i, j, k);
                double V = volume(g, i, j, k);
                double t = T[c];
                double inv_fc = f->cV * rho[c] / (4.0 * OG_A * t * t * t) + 1.0; /* 1/f_c, Eq. 9 */
                double m = V * inv_fc / f->dt;
                double sumw = wr[c] + wt[c] + wp[c];
                if (i > 0) sumw += wr[cidx(g, i - 1, j, k)];
                if (j > 0) sumw += wt[cidx(g, i, j - 1, k)];
                if (np > 1) sumw += wp[cidx(g, i, j, (k + np - 1) % np)];
                d[c] = m + sumw;
                double src = V * (q[c] + (Q ? Q[c] : 0.0));
                b[c] = m * En[c] + src + (i == nr - 1 ? wr[c] * Eb : 0.0);
                s[c] = 1.0 / sqrt(d[c]);
                bhat[c] = s[c] * b[c];
            }

#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < np; k++)
        for (int j = 0; j < nt; j++)
            for (int i = 0; i < nr; i++) {
                long c = cidx(g, i, j, k);
                ahat[c] = (i + 1 < nr) ? -wr[c] * s[c] * s[cidx(g, i + 1, j, k)] : 0.0;
                ahat[n + c] = (j + 1 < nt) ? -wt[c] * s[c] * s[cidx(g, i, j + 1, k)] : 0.0;
                ahat[2 * n + c] = (np > 1) ? -wp[c] * s[c] * s[cidx(g, i, j, (k + 1) % np)] : 0.0;
            }
    free(chi);
}

/* y = Ahat x for the Jacobi-scaled operator (unit diagonal, 7-point stencil). */
void og_spmv(const og_grid *g, const double *ahat, const double *x, double *y)
{
    int nr = g->nr, nt = g->nt, np = g->np;
    long n = (long)nr * nt * np;
    const double *ar = ahat, *at = ahat + n, *ap = ahat + 2 * n;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < np; k++)
        for (int j = 0; j < nt; j++)
            for (int i = 0; i < nr; i++) {
                long c = cidx(g, i, j, k);
                double v = x[c];
                if (i + 1 < nr) v += ar[c] * x[cidx(g, i + 1, j, k)];
                if (i > 0) v += ar[cidx(g, i - 1, j, k)] * x[cidx(g, i - 1, j, k)];
                if (j + 1 < nt) v += at[c] * x[cidx(g, i, j + 1, k)];
                if (j > 0) v += at[cidx(g, i, j - 1, k)] * x[cidx(g, i, j - 1, k)];
                if (np > 1) {
                    long kp = cidx(g, i, j, (k + 1) % np), km = cidx(g, i, j, (k + np - 1) % np);
                    v += ap[c] * x[kp];
                    v += ap[km] * x[km];
                }
                y[c] = v;
            }
}

static double dot(long n, const double *a, const double *b)
{
#ifdef _OPENMP
    /* fixed blocks, block sums added in block order (independent of the thread count) */
    const long B = 4096, nb = (n + B - 1) / B;
    double *part = (double *)malloc(sizeof(double) * (nb > 0 ? nb : 1));
#pragma omp parallel for schedule(static)
    for (long m = 0; m < nb; m++) {
        double s = 0.0;
        long e = (m + 1) * B < n ? (m + 1) * B : n;
        for (long i = m * B; i < e; i++) s += a[i] * b[i];
        part[m] = s;
    }
    double s = 0.0;
    for (long m = 0; m < nb; m++) s += part[m];
    free(part);
    return s;
#else
    double s = 0.0;
    for (long i = 0; i < n; i++) s += a[i] * b[i];
    return s;
#endif
}

/* ||bhat - Ahat y|| / ||bhat|| (reading R7). */
double og_relres(const og_grid *g, const double *ahat, const double *bhat, const double *y)
{
    long n = (long)g->nr * g->nt * g->np;
    double *t = (double *)malloc(sizeof(double) * n);
    og_spmv(g, ahat, y, t);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; c++) t[c] = bhat[c] - t[c];
    double rr = dot(n, t, t), bb = dot(n, bhat, bhat);
    free(t);
    return bb > 0 ? sqrt(rr / bb) : sqrt(rr);
}

/*
 * Conjugate gradients on the Jacobi-scaled system (the implicit Krylov solve of the
 * "generalized minimal residual method" section; the scaled operator is symmetric
 * positive definite, so CG is the Krylov method that applies).  y holds the start
 * guess on entry.  The true residual is recomputed every 50 iterations and whenever
 * the recurrence residual meets the tolerance.  Returns 0 when converged, 1 if
 * max_iter was reached.
 */
int og_cg(const og_grid *g, const double *ahat, const double *bhat, double *y,
          double tol, int max_iter, int *iters, double *relres)
{
    long n = (long)g->nr * g->nt * g->np;
    double *r = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *qv = (double *)malloc(sizeof(double) * n);
    double bn = sqrt(dot(n, bhat, bhat));
    if (bn == 0.0) bn = 1.0;
    og_spmv(g, ahat, y, qv);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; c++) { r[c] = bhat[c] - qv[c]; p[c] = r[c]; }
    double rr = dot(n, r, r);
    int it = 0, status = 1;
    double res = sqrt(rr) / bn;
    if (res <= tol) status = 0;
    while (status && it < max_iter) {
        it++;
        og_spmv(g, ahat, p, qv);
        double alpha = rr / dot(n, p, qv);
#pragma omp parallel for schedule(static)
        for (long c = 0; c < n; c++) { y[c] += alpha * p[c]; r[c] -= alpha * qv[c]; }
        double rr1 = dot(n, r, r);
        if (it % 50 == 0 || sqrt(rr1) / bn <= tol) {
            res = og_relres(g, ahat, bhat, y);
            if (res <= tol) { status = 0; break; }
        } else
            res = sqrt(rr1) / bn;
        double beta = rr1 / rr;
        rr = rr1;
#pragma omp parallel for schedule(static)
        for (long c = 0; c < n; c++) p[c] = r[c] + beta * p[c];
    }
    if (status) res = og_relres(g, ahat, bhat, y);
    if (iters) *iters = it;
    if (relres) *relres = res;
    free(r); free(p); free(qv);
    return status;
}

/*
 * Restarted GMRES(m) on the Jacobi-scaled system (the "generalized minimal residual
 * method" section: the iterate of step i minimises the residual norm over y0 + K_i
 * with K_i = span{r0, A r0, ..., A^(i-1) r0}; after m steps the method starts again
 * from the last iterate).  Arnoldi with modified Gram-Schmidt builds an orthonormal
 * basis V and the Hessenberg matrix H (A V_i = V_(i+1) H_i); Givens rotations reduce H
 * to triangular form, so |g_(i+1)| is the residual norm of the least-squares solution;
 * at a restart or convergence y += V_i H_i^-1 g_i and the true residual is recomputed.
 * Returns 0 when converged, 1 if max_iter inner steps were reached.
 */
int og_gmres(const og_grid *g, const double *ahat, const double *bhat, double *y, int m,
             double tol, int max_iter, int *iters, double *relres)
{
    long n = (long)g->nr * g->nt * g->np;
    if (m < 1) m = 1;
    double *V = (double *)malloc(sizeof(double) * (size_t)n * (m + 1));
    double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double));  /* H[i * m + j] */
    double *cs = (double *)malloc(sizeof(double) * m);
    double *sn = (double *)malloc(sizeof(double) * m);
    double *gv = (double *)malloc(sizeof(double) * (m + 1));
    double *w = (double *)malloc(sizeof(double) * n);
    double bn = sqrt(dot(n, bhat, bhat));
    if (bn == 0.0) bn = 1.0;
    int it = 0, status = 1;
    double res = og_relres(g, ahat, bhat, y);
    if (res <= tol) status = 0;
    while (status && it < max_iter) {
        /* r0 = b - A y, v_0 = r0 / beta */
        og_spmv(g, ahat, y, w);
        for (long c = 0; c < n; c++) w[c] = bhat[c] - w[c];
        double beta = sqrt(dot(n, w, w));
        if (beta == 0.0) { status = 0; res = 0.0; break; }
        for (long c = 0; c < n; c++) V[c] = w[c] / beta;
        for (int i = 0; i <= m; i++) gv[i] = 0.0;
        gv[0] = beta;
        int k = 0;
        for (int j = 0; j < m && it < max_iter; j++) {
            it++;
            og_spmv(g, ahat, V + (size_t)j * n, w);
            for (int i = 0; i <= j; i++) {          /* modified Gram-Schmidt */
                double h = dot(n, w, V + (size_t)i * n);
                H[i * m + j] = h;
                for (long c = 0; c < n; c++) w[c] -= h * V[(size_t)i * n + c];
            }
            double hn = sqrt(dot(n, w, w));
            H[(j + 1) * m + j] = hn;
            if (hn > 0.0)
                for (long c = 0; c < n; c++) V[(size_t)(j + 1) * n + c] = w[c] / hn;
            for (int i = 0; i < j; i++) {            /* previous rotations on column j */
                double a = H[i * m + j], b = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * b;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            double a = H[j * m + j], b = H[(j + 1) * m + j];
            double d = sqrt(a * a + b * b);
            cs[j] = d > 0.0 ? a / d : 1.0;
            sn[j] = d > 0.0 ? b / d : 0.0;
            H[j * m + j] = d;
            H[(j + 1) * m + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            k = j + 1;
            if (fabs(gv[j + 1]) / bn <= tol || hn == 0.0) break;
        }
        /* y += V_k z with H_k z = g_k (back substitution) */
        for (int i = k - 1; i >= 0; i--) {
            double t = gv[i];
            for (int l = i + 1; l < k; l++) t -= H[i * m + l] * gv[l];
            gv[i] = t / H[i * m + i];
        }
        for (int i = 0; i < k; i++)
            for (long c = 0; c < n; c++) y[c] += gv[i] * V[(size_t)i * n + c];
        res = og_relres(g, ahat, bhat, y);
        if (res <= tol) status = 0;
    }
    if (iters) *iters = it;
    if (relres) *relres = res;
    free(V); free(H); free(cs); free(sn); free(gv); free(w);
    return status;
}

/* Dense Cholesky solve of the scaled system for tiny grids (n <= 4096). */
int og_dense_solve(const og_grid *g, const double *ahat, const double *bhat, double *y)
{
    long n = (long)g->nr * g->nt * g->np;
    if (n > 4096) return -1;
    double *A = (double *)calloc((size_t)(n * n), sizeof(double));
    double *e = (double *)calloc((size_t)n, sizeof(double));
    double *col = (double *)malloc(sizeof(double) * n);
    for (long jj = 0; jj < n; jj++) { /* column jj = Ahat e_jj */
        e[jj] = 1.0;
        og_spmv(g, ahat, e, col);
        e[jj] = 0.0;
        for (long ii = 0; ii < n; ii++) A[ii * n + jj] = col[ii];
    }
    int status = 0;
    for (long jj = 0; jj < n && !status; jj++) { /* A = L L^T, L stored in the lower part */
        double s = A[jj * n + jj];
        for (long m = 0; m < jj; m++) s -= A[jj * n + m] * A[jj * n + m];
        if (!(s > 0.0)) { status = 2; break; }
        double ljj = sqrt(s);
        A[jj * n + jj] = ljj;
        for (long ii = jj + 1; ii < n; ii++) {
            double t = A[ii * n + jj];
            for (long m = 0; m < jj; m++) t -= A[ii * n + m] * A[jj * n + m];
            A[ii * n + jj] = t / ljj;
        }
    }
    if (!status) {
        for (long ii = 0; ii < n; ii++) { /* L z = b */
            double t = bhat[ii];
            for (long m = 0; m < ii; m++) t -= A[ii * n + m] * y[m];
            y[ii] = t / A[ii * n + ii];
        }
        for (long ii = n - 1; ii >= 0; ii--) { /* L^T y = z */
            double t = y[ii];
            for (long m = ii + 1; m < n; m++) t -= A[m * n + ii] * y[m];
            y[ii] = t / A[ii * n + ii];
        }
    }
    free(A); free(e); free(col);
    return status;
}

/* ------------------------------------------------- Newton on Eq. (16) (R8) */

/* g(T) = a T^4 - E - S / kappa_P(T), the residual of Eq. (16); *dg = g'(T). */
static double g16(const og_opac *op, double E, double S, double t, double *dg)
{
    double slope;
    double kp = loglog(op, op->kapP, t, &slope);
    if (dg) *dg = 4.0 * OG_A * t * t * t + (S / kp) * slope / t;
    return OG_A * t * t * t * t - E - S / kp;
}

/* Solves a T^4 = E + S / kappa_P(T) per cell (R8); T holds T^n on entry (start value).
 * Bracket: lo = (E/a)^(1/4) where g <= 0; walk the table nodes upward from lo until g
 * turns non-negative (beyond the last node kappa_P is constant, so doubling T ends
 * the walk).  This isolates the smallest root in one table segment. */
void og_newton(const og_grid *g, const og_opac *op, const double *E, const double *S, double *T)
{
    long n = (long)g->nr * g->nt * g->np;
#pragma omp parallel for schedule(dynamic, 4096)
    for (long c = 0; c < n; c++) {
        double e = E[c], s = S[c];
        double lo = pow(e / OG_A, 0.25), hi = -1.0;
        for (int m = 0; m < op->nT; m++) {
            if (op->T[m] <= lo) continue;
            if (g16(op, e, s, op->T[m], NULL) >= 0.0) { hi = op->T[m]; break; }
            lo = op->T[m];
        }
        if (hi < 0.0) {
            hi = 2.0 * lo;
            for (int m = 0; m < 200 && g16(op, e, s, hi, NULL) < 0.0; m++) { lo = hi; hi = 2.0 * hi; }
        }
        double t = T[c];
        if (!(t >= lo)) t = lo;
        if (t > hi) t = hi;
        for (int it = 0; it < 50; it++) {
            double dg;
            double gv = g16(op, e, s, t, &dg);
            if (gv == 0.0) break;
            if (gv < 0.0) lo = t; else hi = t;
            double step = gv / dg;
            double tn = t - step;
            if (fabs(step) <= 1e-14 * t) { t = tn; break; }
            if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi); /* safeguard: bisect */
            t = tn;
        }
        T[c] = t;
    }
}

/* --------------------------------------------- radiative force, Eqs. (27)-(36) */

/*
 * f[4n]: component 0 is the stellar force density q/c (Eq. 36 in the cell-integrated
 * form of Eq. 33); components 1-3 are the thermal force kappa_R rho F / c (Eq. 27)
 * along r, theta, phi with the FLD flux F = -D grad E (Eq. 10) at faces, averaged over
 * the two faces of each direction (R9).  w are the unscaled outward weights written by
 * og_assemble (w / A = D / ds at that face); chi uses kappa_R(T) rho with the T the
 * coefficients were lagged at.
 */
void og_force(const og_grid *g, const og_opac *op, const og_fld *f, const double *rho,
              const double *T, const double *w, const double *E, const double *q, double *out)
{
    int nr = g->nr, nt = g->nt, np = g->np;
    long n = (long)nr * nt * np;
    const double *wr = w, *wt = w + n, *wp = w + 2 * n;
    double Eb = OG_A * pow(f->Tbc, 4);
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < np; k++)
        for (int j = 0; j < nt; j++)
            for (int i = 0; i < nr; i++) {
                long c = cidx(g, i, j, k);
                double chi = og_kappa_R(op, T[c]) * rho[c];
                double Fo, Fi;
                Fo = (i + 1 < nr) ? -wr[c] / area_r(g, i + 1, j, k) * (E[cidx(g, i + 1, j, k)] - E[c])
                                  : -wr[c] / area_r(g, nr, j, k) * (Eb - E[c]);
                Fi = (i > 0) ? -wr[cidx(g, i - 1, j, k)] / area_r(g, i, j, k) * (E[c] - E[cidx(g, i - 1, j, k)]) : 0.0;
                double fr = chi / OG_C * 0.5 * (Fi + Fo);
                Fo = (j + 1 < nt) ? -wt[c] / area_t(g, i, j + 1, k) * (E[cidx(g, i, j + 1, k)] - E[c]) : 0.0;
                Fi = (j > 0) ? -wt[cidx(g, i, j - 1, k)] / area_t(g, i, j, k) * (E[c] - E[cidx(g, i, j - 1, k)]) : 0.0;
                double ft = chi / OG_C * 0.5 * (Fi + Fo);
                double fp = 0.0;
                if (np > 1) {
                    long kp = cidx(g, i, j, (k + 1) % np), km = cidx(g, i, j, (k + np - 1) % np);
                    Fo = -wp[c] / area_p(g, i, j) * (E[kp] - E[c]);
                    Fi = -wp[km] / area_p(g, i, j) * (E[c] - E[km]);
                    fp = chi / OG_C * 0.5 * (Fi + Fo);
                }
                out[c] = q[c] / OG_C;
                out[n + c] = fr;
                out[2 * n + c] = ft;
                out[3 * n + c] = fp;
            }
}

/* ------------------------------------- Rosseland optical depth, Fig. 8 diagnostic */

/*
 * The thermal-emission optical depth of Sect. "The Flux Limited Diffusion
 * approximation" (Fig. 8): tau_R(r) = sum of kappa_R(T) rho dr over the cells between r
 * and the outer edge, integrated inward along each radial ray.  tau[(N_r + 1) per
 * column] at the radial faces: tau at r_out is 0 and tau[i] = tau[i + 1] +
 * kappa_R(T_i) rho_i (r_{i+1} - r_i).
 */
void og_tau_rosseland(const og_grid *g, const og_opac *op, const double *rho, const double *T, double *tau)
{
    int nr = g->nr;
    for (int k = 0; k < g->np; k++)
        for (int j = 0; j < g->nt; j++) {
            double *t = tau + (long)(nr + 1) * (j + (long)g->nt * k);
            t[nr] = 0.0;
            for (int i = nr - 1; i >= 0; i--) {
                long c = cidx(g, i, j, k);
                t[i] = t[i + 1] + og_kappa_R(op, T[c]) * rho[c] * (g->rf[i + 1] - g->rf[i]);
            }
        }
}

/* ------------------------------------------------------ one step (Fig. 1) */

/*
 * The main-loop body of Fig. 1: irradiation F^n(T^n) (ray trace) -> E^n(T^n, F^n)
 * (Eq. 16) -> implicit FLD E^{n+1} (Eq. 15) -> Newton T^{n+1} (Eq. 16), plus the
 * radiative force.  T is T^n on entry and T^{n+1} on exit; E receives E^{n+1};
 * f (4n, may be NULL) receives the force.  dense != 0 uses the Cholesky solve.
 * Returns the solver status.
 */
int og_step(const og_grid *g, const og_opac *op, const og_star *st, const og_fld *f,
            const double *rho, double *T, double *E, double *fout, double tol, int max_iter,
            int dense, int *iters, double *relres)
{
    /* dense: 0 = CG, 1 = dense Cholesky, 2 = no diffusion: the pure-absorption runs of
     * the run table, where the thermal radiation field is never transported and stays at
     * the background a T_bc^4 of the initial state, so Eq. 16 balances the absorbed
     * stellar power against re-emission cell by cell */
    long n = (long)g->nr * g->nt * g->np;
    double *q = (double *)malloc(sizeof(double) * n), *S = (double *)malloc(sizeof(double) * n);
    double *En = (double *)malloc(sizeof(double) * n), *w = (double *)malloc(sizeof(double) * 3 * n);
    double *d = (double *)malloc(sizeof(double) * n), *b = (double *)malloc(sizeof(double) * n);
    double *s = (double *)malloc(sizeof(double) * n), *ah = (double *)malloc(sizeof(double) * 3 * n);
    double *bh = (double *)malloc(sizeof(double) * n), *y = (double *)malloc(sizeof(double) * n);
    double *Tn = (double *)malloc(sizeof(double) * n);
    memcpy(Tn, T, sizeof(double) * n);
    og_raytrace(g, op, st, rho, Tn, q, S, NULL, NULL);
    og_energy(g, op, f, Tn, S, En);
    og_assemble(g, op, f, rho, Tn, En, q, NULL, w, d, b, s, ah, bh);
    for (long c = 0; c < n; c++) y[c] = En[c] / s[c];
    int status;
    if (dense == 2) {
        status = 0;
        if (iters) *iters = 0;
        if (relres) *relres = 0.0;
    } else if (dense) {
        status = og_dense_solve(g, ah, bh, y);
        if (iters) *iters = 0;
        if (relres) *relres = og_relres(g, ah, bh, y);
    } else
        status = og_cg(g, ah, bh, y, tol, max_iter, iters, relres);
    for (long c = 0; c < n; c++) E[c] = dense == 2 ? OG_A * pow(f->Tbc, 4) : s[c] * y[c];
    og_newton(g, op, E, S, T);
    if (fout) og_force(g, op, f, rho, Tn, w, E, q, fout);
    free(q); free(S); free(En); free(w); free(d); free(b); free(s); free(ah); free(bh); free(y); free(Tn);
    return status;
}

/*
 * The main iteration of Fig. 1 run to a steady state: steps of og_step (mode as its
 * `dense` argument) until the largest relative temperature change of a step is below
 * tol_change (the run setup stops at 0.01 %) or max_steps.  Returns the number of steps
 * taken; *last_change is the change of the last step.
 */
int og_relax(const og_grid *g, const og_opac *op, const og_star *st, const og_fld *f, const double *rho,
             double *T, double *E, int mode, double tol, int max_iter, int max_steps, double tol_change,
             double *last_change)
{
    long n = (long)g->nr * g->nt * g->np;
    double *Told = (double *)malloc(sizeof(double) * n);
    int k = 0;
    double ch = INFINITY;
    while (k < max_steps) {
        memcpy(Told, T, sizeof(double) * n);
        og_step(g, op, st, f, rho, T, E, NULL, tol, max_iter, mode, NULL, NULL);
        k++;
        ch = 0.0;
        for (long c = 0; c < n; c++) {
            double r = fabs(T[c] - Told[c]) / Told[c];
            if (r > ch) ch = r;
        }
        if (ch < tol_change) break;
    }
    if (last_change) *last_change = ch;
    free(Told);
    return k;
}

/*
 * Gray irradiation (Eqs. 18, 19): one bin with the stellar flux sigma T_*^4 = sum of the
 * bin fluxes F_b and the opacity kappa_P(T_*), the Planck mean at the stellar
 * temperature, here the F_b-weighted mean of the tabulated bin opacities at each table
 * temperature (so the dust-temperature dependence of the table, e.g. sublimation, is
 * kept).  kappa_gray[k] for the n_T table temperatures; returns sum_b F_b.
 */
double og_gray_table(const og_opac *op, const double *F, double *kappa_gray)
{
    double Fs = 0.0;
    for (int b = 0; b < op->nnu; b++) Fs += F[b];
    for (int k = 0; k < op->nT; k++) {
        double t = 0.0;
        for (int b = 0; b < op->nnu; b++) t += op->kap[k * op->nnu + b] * F[b];
        kappa_gray[k] = t / Fs;
    }
    return Fs;
}

/* Threads the oracle's parallel loops use (1 in the serial build). */
int og_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
