// Internal declarations of librtmi: device helpers, the context, kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/rt.h"

namespace rt {

// CGS constants (CODATA 2018).
constexpr double kC = 2.99792458e10;
constexpr double kSigma = 5.670374419e-5;
constexpr double kA = 4.0 * kSigma / kC;  // radiation constant, sigma = a c / 4 (Eq. 18)
constexpr double kH = 6.62607015e-27;
constexpr double kBoltz = 1.380649e-16;

constexpr int kMaxNu = 64;    // bins per ray trace wavefront (lanes = bins)
constexpr int kMaxT = 128;    // opacity-table temperatures held in LDS

// Grid dimensions; cell c = i + nr (j + nt k).
struct Dims {
    int nr, nt, np;
    long n;       // nr * nt * np
    long plane;   // nr * nt
    int rev = 0;  // Krylov kernels: sweep the rows in reverse order (see for_segments)
};

// 1-D geometry factors on the device (products of them give every volume, area and
// centre distance of the spherical-polar cells).
struct Geo {
    const double *rf;      // [nr+1] radial faces
    const double *rf2;     // [nr+1] r_face^2
    const double *rc;      // [nr]   radial centres (arithmetic midpoints)
    const double *dr;      // [nr]   r_+ - r_-
    const double *shell;   // [nr]   r_+^3 - r_-^3
    const double *vol_r;   // [nr]   (r_+^3 - r_-^3) / 3
    const double *hr2;     // [nr]   (r_+^2 - r_-^2) / 2
    const double *dsr;     // [nr]   centre distance to the next cell (last: ghost centre)
    const double *dcos;    // [nt]   cos(th_-) - cos(th_+)
    const double *sinf;    // [nt+1] sin(th_face)
    const double *dth;     // [nt]   th_+ - th_-
    const double *dtc;     // [nt]   tc[j+1] - tc[j] (last unused)
    const double *sinc;    // [nt]   sin(tc)
    const double *dph;     // [np]   ph_+ - ph_-
    const double *dpc;     // [np]   centre distance to the next cell, periodic
};

// Opacity table on the device.
struct Opac {
    int nT, nnu;
    int kconst;          // rows 0 .. kconst-1 of kap are identical (kappa_nu independent of T there)
    const double *T;     // [nT]
    const double *kap;   // [nT][nnu]
    const double *kP;    // [nT] Planck means
    const double *kR;    // [nT] Rosseland means
    const double *lnT;   // [nT]
    const double *lnP;   // [nT]
    const double *lnR;   // [nT]
};

// ---------------------------------------------------------------- device helpers

// Largest node k in [0, nT-2] with T[k] <= t (caller has handled t outside the table).
__device__ __forceinline__ int find_node(const double *__restrict__ Tt, int nT, double t)
{
    int lo = 0, hi = nT - 1;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (Tt[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// Node and linear weight of t in the table (kappa_nu is linear in T), clamped.
__device__ __forceinline__ void lin_node(const double *__restrict__ Tt, int nT, double t, int &k, double &w)
{
    if (t <= Tt[0]) { k = 0; w = 0.0; return; }
    if (t >= Tt[nT - 1]) { k = nT - 2; w = 1.0; return; }
    k = find_node(Tt, nT, t);
    w = (t - Tt[k]) / (Tt[k + 1] - Tt[k]);
}

// Mean opacity interpolated log-log in T; *slope = d ln kappa / d ln T (0 when clamped).
__device__ __forceinline__ double mean_opacity(const double *__restrict__ Tt, const double *__restrict__ lnT,
                                               const double *__restrict__ tab, const double *__restrict__ lnY,
                                               int nT, double t, double *slope)
{
    if (t <= Tt[0]) { if (slope) *slope = 0.0; return tab[0]; }
    if (t >= Tt[nT - 1]) { if (slope) *slope = 0.0; return tab[nT - 1]; }
    int k = find_node(Tt, nT, t);
    double l0 = lnT[k], l1 = lnT[k + 1];
    double lw = (log(t) - l0) / (l1 - l0);
    if (slope) *slope = (lnY[k + 1] - lnY[k]) / (l1 - l0);
    return exp((1.0 - lw) * lnY[k] + lw * lnY[k + 1]);
}

// FLD diffusion coefficient at a face between cells a and b: Eqs. (11)-(13) with
// (kappa_R rho) and E averaged over the two cells and R from the normal difference;
// above R = 1e100 the limiter (2+R)/(6+3R+R^2) is replaced by its limit 1/R.
__device__ __forceinline__ double face_D(double chi_a, double chi_b, double Ea, double Eb, double ds)
{
    double chi = 0.5 * (chi_a + chi_b);
    double Ef = 0.5 * (Ea + Eb);
    double R = fabs(Eb - Ea) / (ds * chi * Ef);
    double lam = R < 1e100 ? (2.0 + R) / (6.0 + 3.0 * R + R * R) : 1.0 / R;
    return kC * lam / chi;
}

// e = exp(-x) and m = 1 - exp(-x) for x >= 0 from one range reduction: x = k ln2 + r
// with |r| <= ln2/2 (Cody-Waite split of ln2), p = expm1(u), u = -r, as u q(u) with q the
// degree-10 polynomial closest to expm1(u)/u in relative error on that interval (Remez
// exchange, csrc/expm1_minimax.py: error 1.8e-17), then e = 2^-k (1 + p) and
// m = (1 - 2^-k) - 2^-k p, which keeps full relative accuracy for small and large x
// (within 0.7 ulp for e and 1.01 ulp for m).
// x is first clamped to 2000 (e underflows to 0 long before); the clamp is a minimum,
// so a NaN x gives x = 2000.
__device__ __forceinline__ void exp_pair(double x, double &e, double &m)
{
    constexpr double kInvLn2 = 1.4426950408889634074;
    constexpr double kLn2Hi = 6.93147180369123816490e-01;
    constexpr double kLn2Lo = 1.90821492927058770002e-10;
    constexpr double kRound = 6755399441055744.0;  // 1.5 * 2^52: adding it rounds to an integer
    x = fmin(x, 2000.0);
    // -k = rint(-x / ln2), as t = -x / ln2 + 1.5 * 2^52 rounded once: the low word of t is
    // -k as a 32-bit integer (|k| < 2^31) and t - 1.5 * 2^52 is -k exactly
    const double t = fma(x, -kInvLn2, kRound);
    const double nk = t - kRound;
    double r = fma(nk, kLn2Hi, x);
    r = fma(nk, kLn2Lo, r);
    double u = -r;
    // BEGIN expm1 minimax: q(u) coefficients, highest degree first
    double p = 2.505209761119569e-08;
    p = fma(p, u, 2.762626294187125e-07);
    p = fma(p, u, 2.755741478642639e-06);
    p = fma(p, u, 2.480150460177586e-05);
    p = fma(p, u, 0.00019841269707470595);
    p = fma(p, u, 0.001388888893225918);
    p = fma(p, u, 0.008333333333397832);
    p = fma(p, u, 0.041666666666573905);
    p = fma(p, u, 0.16666666666666563);
    p = fma(p, u, 0.5000000000000006);
    p = fma(p, u, 1.0);
    // END expm1 minimax
    p = p * u;                                     // expm1(u)
    double s = ldexp(1.0, __double2loint(t));
    e = fma(s, p, s);
    // 1 - e = -(s p + (s - 1)): s - 1 is exact (k >= 0 since x >= 0), so one rounding;
    // for k = 0 it is -p exactly
    m = -fma(s, p, s - 1.0);
}

// Orders LDS traffic between the lanes of one wavefront.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double readlane_d(double v, int lane)
{
    int2 t = *reinterpret_cast<int2 *>(&v);
    t.x = __builtin_amdgcn_readlane(t.x, lane);
    t.y = __builtin_amdgcn_readlane(t.y, lane);
    return *reinterpret_cast<double *>(&t);
}

// ------------------------------------------------------------------- context

// Krylov scalars kept in device memory and updated by the last block of each
// reduction kernel; the host reads them back only to poll convergence.
struct DevScalars {
    double rr;       // r.r of the current residual (recurrence)
    double pq;       // p.q
    double alpha, beta;
    double thresh2;  // stop when rr <= thresh2
    double res2;     // last reduction of the residual kernel
    double inv_norm; // 1 / sqrt(res2)
    double change;   // largest relative temperature change of the last main iteration
    double bnorm2;   // ||b^||^2 of the solve (1 when b^ = 0), set on the device by k_solve_init
    int done;
    int iters;
};

struct Net;

// Multigrid preconditioner (k_mg.hip).  Level l of the hierarchy: n = N_r nt np cells;
// operator dg / ar / at / ap (dg null: unit diagonal, the finest level A^), the
// prolongation weights w to level l+1, the phi-line factors (im, cp, q, g per cell,
// rho, kap per (r, theta) line) and the V-cycle's vectors.
struct MgLevel {
    int nt = 0, np = 0;
    long n = 0;
    const float *dg = nullptr, *ar = nullptr, *at = nullptr, *ap = nullptr;
    const float *w = nullptr, *im = nullptr, *cp = nullptr, *q = nullptr, *g = nullptr;
    const float *rho = nullptr, *kap = nullptr;
    float *b = nullptr, *x = nullptr, *x2 = nullptr, *dp = nullptr;
    float *xr = nullptr;  // the level's coarse-correction result (levels 1 .. L)
};

struct MgLevel64 {
    double *dg = nullptr, *ar = nullptr, *at = nullptr, *ap = nullptr, *B = nullptr;
};

// A level with K-cycle steps (two flexible-CG steps per coarse correction): the two
// preconditioned vectors, A z_1 and the device scalars (p.q, alpha, beta); z is null on
// other levels.
struct MgKLevel {
    float *z = nullptr, *p1 = nullptr, *q = nullptr;
    double *ks = nullptr;
};

struct MgHier {
    int nr = 0;
    std::vector<MgKLevel> kl;    // per level (K-cycle buffers where used)
    int kmax = 0;                // levels 1 .. kmax take K-cycle steps in the next cycles
    double *kpart = nullptr;     // K-cycle reduction partials (five per block)
    std::vector<MgLevel> lev;    // 0 .. L (L: one radial line)
    std::vector<MgLevel64> d64;  // levels 1 .. L in float64 (entry l - 1), built by the set-up
    std::vector<float *> dg32, ar32, at32, ap32;                // levels 1 .. L in float32 (entry l - 1)
    std::vector<float *> w, im, cp, q, g, rho, kap;           // levels 0 .. L - 1
    double *B0 = nullptr, *t64a = nullptr, *t64b = nullptr;  // 1 / s, line-factor scratch (n_0 each)
    double *cim = nullptr, *ccp = nullptr, *inv = nullptr;   // coarsest line: factors, inverse (N_r^2)
    double *part = nullptr;                                   // r.z partial sums (one per line-sweep block)
    unsigned *cnt = nullptr;                                  // their completion counter (0 between uses)
    bool ready = false;                                      // set up for the current system
};

// ------------------------------------------------------------------ launchers
void launch_raytrace(const Dims &d, const Opac &op, const Geo &g, const double *F0, double R2,
                     const double *rho, const double *T, double *q, double *S, double *Fface,
                     double *Fnu, hipStream_t st);
size_t raytrace_lds_bytes(int nT, int nr, bool face);
// The two mappings of a column onto a wavefront: lanes on bins (any outputs) and lanes on
// radial cells (q and S; a multiplicative scan per bin).  launch_raytrace picks one.
void launch_raytrace_bins(const Dims &d, const Opac &op, const Geo &g, const double *F0, double R2,
                          const double *rho, const double *T, double *q, double *S, double *Fface,
                          double *Fnu, hipStream_t st);
void launch_raytrace_r(const Dims &d, const Opac &op, const Geo &g, const double *F0, double R2, const double *rho,
                       const double *T, double *q, double *S, hipStream_t st);
bool raytrace_cells_fit(int nr);  // the column fills its 512-cell segments to 90 % or more
void raytrace_r_prepare();
void launch_energy(const Dims &d, const Opac &op, const double *T, const double *S, double Efloor,
                   double *E, hipStream_t st);
void launch_assemble(const Dims &d, const Geo &g, const Opac &op, const double *rho, const double *T,
                     const double *En, const double *q, const double *Q, double cV, double dt,
                     double Eb, double kR_bc, double *chi, double *w, double *s, double *b,
                     double *bhat, double *ahat, float *ahat32, hipStream_t st);
void launch_newton(const Dims &d, const Opac &op, const double *E, const double *S, double *T,
                   hipStream_t st);
void launch_force(const Dims &d, const Geo &g, const double *w, const double *chi, const double *E,
                  const double *q, double Eb, double *f, hipStream_t st);
void launch_scale_mul(long n, const double *s, const double *x, double *y, hipStream_t st);
void launch_scale_div(long n, const double *s, const double *x, double *y, hipStream_t st);
void launch_fill(long n, double v, double *x, hipStream_t st);
// Inward Rosseland optical depth at the radial faces ((N_r + 1) per column).
void launch_tau_rosseland(const Dims &d, const Opac &op, const double *rf, const double *rho, const double *T,
                          double *tau, hipStream_t st);
// Radial-line block-Jacobi preconditioner (k_krylov.hip): Thomas factors of each radial
// row's tridiagonal block, z = M^-1 r with r.z, and one preconditioned CG iteration.
void launch_line_factor(const Dims &d, int nblk, const double *a, double *c, double *im, hipStream_t st);
void launch_line_solve(const Dims &d, int nblk, const double *a, const double *c, const double *im, const double *r,
                       double *z, double *partials, unsigned *counter, DevScalars *sc, int restart, hipStream_t st);
void launch_pcg_line_iter(const Dims &d, int nblk, int nblk_upd, const double *a, const double *lc, const double *lim,
                          double *y, double *r, double *z, double *pold, double *pnew, double *q, double *partials,
                          unsigned *counter, DevScalars *sc, int restart, hipStream_t st, const hipEvent_t *ev);
// Red-black reduced system (k_krylov.hip): half-grid dims, colour split of the operator
// and of vectors, the passes of one product with S = I - B^T B, and one CG iteration on S.
Dims rb_half(const Dims &d);
void launch_rb_split(const Dims &d, const double *a, double *ab, float *ab32, hipStream_t st);
void launch_rb_gather(const Dims &d, const double *x, double *xb, double *xr, hipStream_t st);
void launch_rb_scatter(const Dims &d, const double *xb, const double *xr, double *x, hipStream_t st);
void launch_rb_red_apply(const Dims &dh, int nblk, const double *ab, const double *x, const double *u, double sgn,
                         double *out, hipStream_t st);
void launch_rb_black_apply(const Dims &dh, int nblk, const double *ab, const double *t, const double *u,
                           const double *x, double sgn, double *out, double *partials, unsigned *counter,
                           DevScalars *sc, int restart, hipStream_t st);
// One-workgroup float64 CG on S for at most 2048 black cells (rb_block_cpt > 0): up to
// m iterations, stopping at convergence; false if the grid is too large.
int rb_block_cpt(const Dims &dh);
bool launch_rb_cg_block(const Dims &dh, const double *ab, double *y, double *r, double *p, int m, DevScalars *sc,
                        hipStream_t st);
void launch_rb_iter64(const Dims &dh, int nblk, int nblk_upd, const double *ab, double *y, double *r, double *pold,
                      double *pnew, double *q, double *t, double *partials, unsigned *counter, DevScalars *sc,
                      hipStream_t st, const hipEvent_t *ev);
void launch_rb_iter32(const Dims &dh, int nblk, int nblk_upd, const float *ab, float *x, float *r, float *pold,
                      float *pnew, float *q, float *t, double *partials, unsigned *counter, DevScalars *sc,
                      hipStream_t st, const hipEvent_t *ev);
// max_c |T_c - Told_c| / Told_c into *out (device); partials needs nblk entries.
void launch_max_change(long n, int nblk, const double *T, const double *Told, double *partials,
                       unsigned *counter, double *out, hipStream_t st);
// Krylov kernels: nblk blocks (a multiple of 8) sweeping the rows in windows; the
// CG iteration launches its update kernel with nblk_upd blocks.
void launch_spmv(const Dims &d, int nblk, const double *a, const double *x, double *y, hipStream_t st);
void launch_spmv32(const Dims &d, int nblk, const float *a, const float *x, float *y, hipStream_t st);
// The host's set-up of a float64 CG solve done on the device, after launch_norm2 of b^:
// bnorm2 = res2 (1 when 0), thresh2 = tol2 bnorm2, done = iters = 0, beta = 0.
void launch_solve_init(DevScalars *sc, double tol2, hipStream_t st);
void launch_norm2(const Dims &d, int nblk, const double *x, double *partials, unsigned *counter,
                  DevScalars *sc, hipStream_t st);
void launch_resid(const Dims &d, int nblk, const double *a, const double *b, const double *y,
                  double *r, double *partials, unsigned *counter, DevScalars *sc, int restart, hipStream_t st);
// One CG iteration (direction+operator kernel, then update kernel).  When ev is given,
// ev[0], ev[1], ev[2] are recorded before, between and after the two kernels.
// odd: the parity of the iteration (the direction pass alternates its sweep direction)
void launch_cg_iter64(const Dims &d, int nblk, int nblk_upd, const double *a, double *y, double *r, double *pold,
                      double *pnew, double *q, double *partials, unsigned *counter, DevScalars *sc,
                      hipStream_t st, const hipEvent_t *ev, int odd);
void launch_cg_iter32(const Dims &d, int nblk, int nblk_upd, const float *a, float *x, float *r, float *pold,
                      float *pnew, float *q, double *partials, unsigned *counter, DevScalars *sc,
                      hipStream_t st, const hipEvent_t *ev, int odd);
void launch_reliable(const Dims &d, int nblk, const double *r, float *r32, float *x32, double *partials,
                     unsigned *counter, DevScalars *sc, int restart, hipStream_t st);
void launch_fold(long n, const float *x32, double *y, hipStream_t st);
// GMRES(m): basis inner products (out[i] = V_i . w, i < k, deterministic), w += sign
// sum coef_i V_i, y = s x.  At most kMaxBasis basis vectors.
constexpr int kMaxBasis = 64;
void launch_mdot(const Dims &d, int nblk, const double *V, int k, const double *w, double *partials, double *out,
                 hipStream_t st);
void launch_maxpy(long n, const double *V, int k, const double *coef, double sign, double *w, hipStream_t st);
void launch_scale_into(long n, const double *x, double s, double *y, hipStream_t st);
void launch_d2f(long n, const double *x, float *y, hipStream_t st);
// Multigrid: the level shapes (theta, phi sizes from the finest to one radial line),
// the set-up of a system (float64 Galerkin levels, line factors, coarsest inverse) and
// one cycle on r: z = M_mg r, with rr = r.z and the flexible-CG beta = -(z.qold) / pq
// (0 when restart) written to sc (whose kernels do nothing once sc->done is set).
void mg_shapes(int nt, int np, std::vector<std::pair<int, int>> &out);
void launch_mg_setup(MgHier &h, const double *ahat, const double *s, hipStream_t st);
void launch_mg_vcycle(MgHier &h, const double *r, double *z, const double *qold, float omega, DevScalars *sc,
                      int restart, hipStream_t st);
// The same cycle on a float32 residual, z in float32 (no dot).
void launch_mg_vcycle32(MgHier &h, const float *r, float *z, float omega, DevScalars *sc, hipStream_t st);
void launch_f2d(long n, const float *x, double *y, hipStream_t st);
// The rest of a preconditioned CG iteration once z = M^-1 r and beta are known.
void launch_pcg_dir_upd(const Dims &d, int nblk, int nblk_upd, const double *a, const double *z, double *y, double *r,
                        double *pold, double *pnew, double *q, double *partials, unsigned *counter, DevScalars *sc,
                        hipStream_t st, const hipEvent_t *ev);
// Flexible CG for the learned mode (float32 vectors, float64 dots).
void launch_fcg_dir(const Dims &d, int nblk, const float *a, const float *z, const float *pold, const float *r,
                    float *pnew, float *q, double *partials, unsigned *counter, DevScalars *sc, hipStream_t st);
void launch_fcg_beta(const Dims &d, int nblk, const float *z, const float *q, double *partials, unsigned *counter,
                     DevScalars *sc, hipStream_t st);
void launch_cg_upd32(const Dims &d, int nblk, float *x, const float *p, float *r, const float *q, double *partials,
                     unsigned *counter, DevScalars *sc, hipStream_t st);
void launch_rms_scale(long n, const DevScalars *sc, double *scale, hipStream_t st);
void launch_norm2_rr32(const Dims &d, int nblk, const float *x, double *partials, unsigned *counter,
                       DevScalars *sc, hipStream_t st);

// U-Net kernels (k_unet.hip): bf16 tensors as raw 16-bit values.
namespace nn {
typedef unsigned short bf16;
struct Lv {
    int nr, nt, np;
    long n;
};
bool launch_conv_fwd(const Lv &L, const bf16 *x1, int c1, int up1, const bf16 *x2, int c2, const bf16 *w,
                     const float *b, int cout, int relu, bf16 *y, float *yf, hipStream_t s);
bool launch_conv_bwd_data(const Lv &L, const float *dy, const bf16 *y, int cout, const bf16 *wt, int c1, float *d1,
                          int c2, float *d2, hipStream_t s);
bool launch_conv_bwd_weight(const Lv &L, const float *dy, const bf16 *y, int cout, const bf16 *x1, int c1, int up1,
                            const bf16 *x2, int c2, float *part, float *dw, float *db, hipStream_t s);
long wgrad_part_floats(const Lv &L, int cout, int cin);
// relu(conv(x, w) + b) (16 -> 16) followed by the 1x1 output layer z = wo . h + bo (times
// scale[1] when scale != nullptr), without writing h; bit for bit the two layers' result.
void launch_conv_fwd_head(const Lv &L, const bf16 *x, const bf16 *w, const float *b, const bf16 *wo, const float *bo,
                          const double *scale, float *z, hipStream_t s);
// y = relu(conv(x, w) + b) (16 -> 16, bf16) and yp = its 2x2x2 average pool on the next
// coarser level (16 channels), in one pass; bit for bit the two kernels' results.
void launch_conv_fwd_pool(const Lv &L, const bf16 *x, const bf16 *w, const float *b, bf16 *y, bf16 *yp, hipStream_t s);
void launch_pool(const Lv &Lc, int C, const bf16 *x, bf16 *y, hipStream_t s);
void launch_pool_bwd_add(const Lv &Lf, int C, const float *dyc, float *dxf, hipStream_t s);
void launch_up_bwd(const Lv &Lc, int C, const float *dyf, float *dxc, hipStream_t s);
void launch_out_fwd(long n, const bf16 *x, const bf16 *w, const float *b, const double *scale, float *z,
                    hipStream_t s);
// Layer 0 of a preconditioner application with the scaled residual r as channel 0 of X.
void launch_conv_fwd_in(const Lv &L, const bf16 *X, const float *r, const double *scale, const bf16 *w,
                        const float *b, bf16 *y, hipStream_t s);
void launch_out_bwd(long n, const bf16 *x, const bf16 *w, const float *gz, float *dx, float *part, float *dwb,
                    hipStream_t s);
void launch_features(long n, const double *ahat, bf16 *X, hipStream_t s);
void launch_set_input(long n, const double *r, const double *scale, bf16 *X, hipStream_t s);
void launch_loss(long n, const float *z, const float *e, double *part, double *res, float *gz, hipStream_t s);
void launch_adam(long np_, float *p, const float *g, float *m, float *v, float lr, float b1, float b2, float eps,
                 float c1, float c2, hipStream_t s);
void launch_cast_weights(int taps, int cout, int cin, const float *p, bf16 *w, bf16 *wt, hipStream_t s);
void launch_scaled_f32(long n, const double *r, const double *scale, float *out, hipStream_t s);
void launch_pair(long n, const DevScalars *sc, const double *ystar, const double *y, double *scale, float *e,
                 hipStream_t s);
}  // namespace nn

// Network hooks used by the learned solve and the training set (rt_net.hip).
rt_status net_prepare(rt_net *net, rt_ctx *ctx);                       // workspace + operator features
rt_status net_precond(rt_net *net, rt_ctx *ctx, const float *r, float *z); // z = M(r); uses sc->rr
// Float64 CG on the context's current system from y (in/out), tol and iteration cap.
rt_status solve_fp64_from(rt_ctx *ctx, double tol, int max_iter, double *y, rt_solve_stats *st);
rt_status learned_from(rt_ctx *ctx, rt_net *net, int applies, double *y, rt_solve_stats *st);

}  // namespace rt

struct rt_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    rt::Dims d{};
    int n_nu = 0;
    std::string err;

    // host copies of the problem description
    std::vector<double> h_rf, h_tf, h_pf;
    std::vector<double> h_opac;  // packed copy of the last uploaded table (change detection)
    std::vector<double> h_star;  // packed copy of the last uploaded star
    bool have_opac = false, have_star = false;
    double R_star = 0.0, T_star = 0.0;
    int nT = 0;

    // device memory: one arena per kind, freed at destroy
    std::vector<void *> allocs;
    rt::Geo geo{};
    rt::Opac op{};
    double *F0 = nullptr;  // [n_nu] star flux per bin at R_*

    // step fields
    double *q = nullptr, *S = nullptr, *En = nullptr, *Tn = nullptr;
    // system
    double *w = nullptr, *ahat = nullptr, *s = nullptr, *b = nullptr, *bhat = nullptr, *chi = nullptr;
    float *ahat32 = nullptr;
    bool have_system = false;
    // colour split of ahat / ahat32 for the red-black reduced solves ([2][3][n/2] each),
    // allocated at the first such solve and refreshed once per assembled system
    double *rb_a = nullptr;
    float *rb_a32 = nullptr;
    bool rb_ready = false;
    // radial-line block-Jacobi factors (c, 1/m) and the preconditioned residual z,
    // allocated at the first such solve, factors refreshed once per assembled system
    double *ln_c = nullptr, *ln_im = nullptr, *ln_z = nullptr;
    bool ln_ready = false;
    // HIP graphs of chunks of Krylov iterations (launch-bound small grids): one per
    // (solver kind, start direction buffer, chunk length), replayed on `stream`
    struct GraphEntry {
        int kind;
        const void *pold;
        int m;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    hipStream_t cap_stream = nullptr;  // capture stream (non-blocking, default priority)
    double Eb = 0.0;  // a T_bc^4 of the assembled system
    // Krylov vectors
    double *y = nullptr, *r = nullptr, *p0 = nullptr, *p1 = nullptr, *qv = nullptr, *tmp = nullptr;
    float *r32 = nullptr, *z32 = nullptr, *p32a = nullptr, *p32b = nullptr, *q32 = nullptr, *x32 = nullptr;
    double *nscale = nullptr;  // [2] network input scale and its inverse
    // reductions
    int nblk = 0;             // blocks of the stencil and reduction kernels (multiple of 8)
    int nblk_upd = 0;         // blocks of the streaming update kernels (multiple of 8)
    double *partials = nullptr;
    // GMRES(m) workspace, allocated on first use: basis V (gm_cap vectors of n), the
    // per-block partial inner products and the device copy of small coefficient arrays
    double *gmV = nullptr, *gm_part = nullptr, *gm_coef = nullptr;
    int gm_cap = 0;
    // flexible GMRES: the preconditioned vectors Z (gmz_cap vectors of n)
    double *gmZ = nullptr;
    int gmz_cap = 0;
    unsigned *counter = nullptr;
    rt::DevScalars *sc = nullptr;   // device
    rt::DevScalars *h_sc = nullptr; // pinned host mirror
    hipEvent_t ev[12] = {};

    rt::Net *net_scratch = nullptr;
    // multigrid hierarchy, allocated at the first multigrid solve, set up once per system
    rt::MgHier *mg = nullptr;
    double *mg_z = nullptr;
};
