// Element and stencil kernels of the radiation step around the linear solve:
// E^n from Eq. (16), the FLD assembly of Eqs. (8)-(15), the Newton update of
// Eq. (16) and the radiative force of Eqs. (27)-(36).  All float64; all memory
// access is r-contiguous (one thread per cell, consecutive threads on consecutive
// radii), so every array is streamed once with coalesced loads.
#include "rt_internal.h"

namespace rt {

constexpr int kTB = 256;

__device__ __forceinline__ void cell_ijk(long c, const Dims &d, int &i, int &j, int &k)
{
    i = (int)(c % d.nr);
    long jk = c / d.nr;
    j = (int)(jk % d.nt);
    k = (int)(jk / d.nt);
}

// Fig. 1 "Radiation Energy": E^n = max(a T^4 - S / kappa_P(T), E_floor) (Eq. 16).
__global__ __launch_bounds__(kTB) void k_energy(long n, Opac op, const double *__restrict__ T,
                                                const double *__restrict__ S, double Efloor,
                                                double *__restrict__ E)
{
    long c = (long)blockIdx.x * kTB + threadIdx.x;
    if (c >= n) return;
    double t = T[c];
    double kp = mean_opacity(op.T, op.lnT, op.kP, op.lnP, op.nT, t, nullptr);
    double e = kA * t * t * t * t - S[c] / kp;
    E[c] = e > Efloor ? e : Efloor;
}

// chi = kappa_R(T) rho, the Rosseland extinction entering Eqs. (11) and (13).
__global__ __launch_bounds__(kTB) void k_chi(long n, Opac op, const double *__restrict__ T,
                                             const double *__restrict__ rho, double *__restrict__ chi)
{
    long c = (long)blockIdx.x * kTB + threadIdx.x;
    if (c >= n) return;
    chi[c] = mean_opacity(op.T, op.lnT, op.kR, op.lnR, op.nT, T[c], nullptr) * rho[c];
}

// Outward face weights w = A D / ds of each cell (Eqs. 10-13 at the face).  The radial
// weight of the last cell couples to the Dirichlet ghost (rho_ghost = rho_last, kappa_R
// at T_bc, E = a T_bc^4); the polar weight of the last polar cell is 0 (pole); the
// azimuthal weight couples periodically (0 when there is one azimuthal cell).
__global__ __launch_bounds__(kTB) void k_asm_faces(Dims d, Geo g, const double *__restrict__ chi,
                                                   const double *__restrict__ En,
                                                   const double *__restrict__ rho, double kR_bc,
                                                   double Eb, double *__restrict__ w)
{
    long c = (long)blockIdx.x * kTB + threadIdx.x;
    if (c >= d.n) return;
    int i, j, k;
    cell_ijk(c, d, i, j, k);
    double chic = chi[c], Ec = En[c];
    double wr, wt, wp;
    {
        double ds = g.dsr[i];
        if (i + 1 < d.nr) {
            double A = g.rf2[i + 1] * g.dcos[j] * g.dph[k];
            wr = A * face_D(chic, chi[c + 1], Ec, En[c + 1], ds) / ds;
        } else {
            double A = g.rf2[d.nr] * g.dcos[j] * g.dph[k];
            wr = A * face_D(chic, kR_bc * rho[c], Ec, Eb, ds) / ds;
        }
    }
    if (j + 1 < d.nt) {
        double ds = g.rc[i] * g.dtc[j];
        double A = g.sinf[j + 1] * g.hr2[i] * g.dph[k];
        wt = A * face_D(chic, chi[c + d.nr], Ec, En[c + d.nr], ds) / ds;
    } else {
        wt = 0.0;
    }
    if (d.np > 1) {
        long cn = (k + 1 < d.np) ? c + d.plane : c - (long)(d.np - 1) * d.plane;
        double ds = g.rc[i] * g.sinc[j] * g.dpc[k];
        double A = g.hr2[i] * g.dth[j];
        wp = A * face_D(chic, chi[cn], Ec, En[cn], ds) / ds;
    } else {
        wp = 0.0;
    }
    w[c] = wr;
    w[d.n + c] = wt;
    w[2 * d.n + c] = wp;
}

// Diagonal, right-hand side and Jacobi scale of the backward-Euler system
//   V/(dt f_c) (E - E^n) = sum_f w_f (E_nb - E) + V (q + Q+),  f_c from Eq. (9).
__global__ __launch_bounds__(kTB) void k_asm_diag(Dims d, Geo g, const double *__restrict__ w,
                                                  const double *__restrict__ rho,
                                                  const double *__restrict__ T,
                                                  const double *__restrict__ En,
                                                  const double *__restrict__ q,
                                                  const double *__restrict__ Q, double cV, double dt,
                                                  double Eb, double *__restrict__ s,
                                                  double *__restrict__ b, double *__restrict__ bhat)
{
    long c = (long)blockIdx.x * kTB + threadIdx.x;
    if (c >= d.n) return;
    int i, j, k;
    cell_ijk(c, d, i, j, k);
    const double *wr = w, *wt = w + d.n, *wp = w + 2 * d.n;
    double V = g.vol_r[i] * g.dcos[j] * g.dph[k];
    double t = T[c];
    double inv_fc = cV * rho[c] / (4.0 * kA * t * t * t) + 1.0;
    double m = V * inv_fc / dt;
    double sumw = wr[c] + wt[c] + wp[c];
    if (i > 0) sumw += wr[c - 1];
    if (j > 0) sumw += wt[c - d.nr];
    if (d.np > 1) sumw += wp[(k > 0) ? c - d.plane : c + (long)(d.np - 1) * d.plane];
    double dd = m + sumw;
    double src = V * (q[c] + (Q ? Q[c] : 0.0));
    double bb = m * En[c] + src + (i == d.nr - 1 ? wr[c] * Eb : 0.0);
    double sc = 1.0 / sqrt(dd);
    s[c] = sc;
    b[c] = bb;
    bhat[c] = sc * bb;
}

// Scaled off-diagonals ahat = -w s_c s_nb of the outward faces (0 on boundary faces),
// and their float32 copy for the inner solves of the mixed mode.
__global__ __launch_bounds__(kTB) void k_asm_scale(Dims d, const double *__restrict__ w,
                                                   const double *__restrict__ s,
                                                   double *__restrict__ ahat, float *__restrict__ ahat32)
{
    long c = (long)blockIdx.x * kTB + threadIdx.x;
    if (c >= d.n) return;
    int i, j, k;
    cell_ijk(c, d, i, j, k);
    double sc = s[c];
    double ar = (i + 1 < d.nr) ? -w[c] * sc * s[c + 1] : 0.0;
    double at = (j + 1 < d.nt) ? -w[d.n + c] * sc * s[c + d.nr] : 0.0;
    double ap = 0.0;
    if (d.np > 1) {
        long cn = (k + 1 < d.np) ? c + d.plane : c - (long)(d.np - 1) * d.plane;
        ap = -w[2 * d.n + c] * sc * s[cn];
    }
    ahat[c] = ar;
    ahat[d.n + c] = at;
    ahat[2 * d.n + c] = ap;
    ahat32[c] = (float)ar;
    ahat32[d.n + c] = (float)at;
    ahat32[2 * d.n + c] = (float)ap;
}

// g(T) = a T^4 - E - S / kappa_P(T), the residual of Eq. (16), and g'(T); kappa_P
// interpolated log-log in the table interval k (the caller guarantees T[k] <= t <
// T[k+1], or k = -1 / k = nT - 1 for t below / above the table, where kappa_P is the
// end value).
__device__ __forceinline__ double g16(const Opac &op, double E, double S, double t, int k, double &dg)
{
    double kp, slope = 0.0;
    if (k < 0) kp = op.kP[0];
    else if (k >= op.nT - 1) kp = op.kP[op.nT - 1];
    else {
        const double l0 = op.lnT[k], l1 = op.lnT[k + 1];
        const double lw = (log(t) - l0) / (l1 - l0);
        slope = (op.lnP[k + 1] - op.lnP[k]) / (l1 - l0);
        kp = exp((1.0 - lw) * op.lnP[k] + lw * op.lnP[k + 1]);
    }
    dg = 4.0 * kA * t * t * t + (S / kp) * slope / t;
    return kA * t * t * t * t - E - S / kp;
}

// Table interval of t for g16.
__device__ __forceinline__ int p_interval(const Opac &op, double t)
{
    if (t < op.T[0]) return -1;
    if (t >= op.T[op.nT - 1]) return op.nT - 1;
    return find_node(op.T, op.nT, t);
}

// Newton-Raphson on Eq. (16) per cell, safeguarded by a bracket that isolates the
// smallest root: lo = (E/a)^(1/4) (g <= 0 there), then the table nodes above lo are
// walked until g >= 0 (at a node kappa_P is the tabulated value; past the table it is
// constant, so doubling ends the walk).  The smallest root then lies in one table
// interval (or beyond the table), so every Newton step evaluates kappa_P in a known
// interval.  Iterates from T^n; a step that leaves the bracket is replaced by
// bisection; stops when the Newton step is below 1e-14 T or after 50 iterations.
__global__ __launch_bounds__(kTB) void k_newton(long n, Opac op, const double *__restrict__ E,
                                                const double *__restrict__ S, double *__restrict__ T)
{
    long c = (long)blockIdx.x * kTB + threadIdx.x;
    if (c >= n) return;
    double e = E[c], sv = S[c], dg;
    double lo = pow(e / kA, 0.25), hi = -1.0;
    int m0 = (lo < op.T[0]) ? 0 : (lo >= op.T[op.nT - 1] ? op.nT : find_node(op.T, op.nT, lo) + 1);
    for (int m = m0; m < op.nT; m++) {
        double tm = op.T[m];
        if (tm <= lo) continue;
        if (kA * tm * tm * tm * tm - e - sv / op.kP[m] >= 0.0) { hi = tm; break; }
        lo = tm;
    }
    if (hi < 0.0) {
        hi = 2.0 * lo;
        for (int m = 0; m < 200 && g16(op, e, sv, hi, op.nT - 1, dg) < 0.0; m++) { lo = hi; hi = 2.0 * hi; }
    }
    // the interval of the bracket: lo and hi are adjacent walk points, so [lo, hi) lies
    // in the table interval of lo (or beyond the table)
    const int k = p_interval(op, lo);
    double t = T[c];
    if (!(t >= lo)) t = lo;
    if (t > hi) t = hi;
    for (int it = 0; it < 50; it++) {
        const int kt = (t >= hi && k >= 0 && k < op.nT - 1) ? p_interval(op, t) : k;
        double gv = g16(op, e, sv, t, kt, dg);
        if (gv == 0.0) break;
        if (gv < 0.0) lo = t; else hi = t;
        double step = gv / dg;
        double tn = t - step;
        if (fabs(step) <= 1e-14 * t) { t = tn; break; }
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        t = tn;
    }
    T[c] = t;
}

// Radiative force density per cell (Eq. 27): f0 = q / c (stellar, Eq. 36 in the cell-
// integrated form of Eq. 33); f1..f3 = chi / c times the mean of the two face fluxes
// F = -(w / A)(E_nb - E) (FLD flux of Eq. 10 with the lagged D of the system).
__global__ __launch_bounds__(kTB) void k_force(Dims d, Geo g, const double *__restrict__ w,
                                               const double *__restrict__ chi,
                                               const double *__restrict__ E,
                                               const double *__restrict__ q, double Eb,
                                               double *__restrict__ f)
{
    long c = (long)blockIdx.x * kTB + threadIdx.x;
    if (c >= d.n) return;
    int i, j, k;
    cell_ijk(c, d, i, j, k);
    const double *wr = w, *wt = w + d.n, *wp = w + 2 * d.n;
    double Ec = E[c], x = chi[c] / kC;
    double Fo, Fi;
    Fo = (i + 1 < d.nr) ? -wr[c] / (g.rf2[i + 1] * g.dcos[j] * g.dph[k]) * (E[c + 1] - Ec)
                        : -wr[c] / (g.rf2[d.nr] * g.dcos[j] * g.dph[k]) * (Eb - Ec);
    Fi = (i > 0) ? -wr[c - 1] / (g.rf2[i] * g.dcos[j] * g.dph[k]) * (Ec - E[c - 1]) : 0.0;
    double fr = x * 0.5 * (Fi + Fo);
    Fo = (j + 1 < d.nt) ? -wt[c] / (g.sinf[j + 1] * g.hr2[i] * g.dph[k]) * (E[c + d.nr] - Ec) : 0.0;
    Fi = (j > 0) ? -wt[c - d.nr] / (g.sinf[j] * g.hr2[i] * g.dph[k]) * (Ec - E[c - d.nr]) : 0.0;
    double ft = x * 0.5 * (Fi + Fo);
    double fp = 0.0;
    if (d.np > 1) {
        long kp = (k + 1 < d.np) ? c + d.plane : c - (long)(d.np - 1) * d.plane;
        long km = (k > 0) ? c - d.plane : c + (long)(d.np - 1) * d.plane;
        double A = g.hr2[i] * g.dth[j];
        Fo = -wp[c] / A * (E[kp] - Ec);
        Fi = -wp[km] / A * (Ec - E[km]);
        fp = x * 0.5 * (Fi + Fo);
    }
    f[c] = q[c] / kC;
    f[d.n + c] = fr;
    f[2 * d.n + c] = ft;
    f[3 * d.n + c] = fp;
}

// y = s * x (E = s y) and y = x / s (start guess y0 = E^n / s).
// Rosseland optical depth of the thermal emission integrated inward from the outer edge
// (the Fig. 8 diagnostic): tau[i] = sum over cells i' >= i of kappa_R(T) rho dr at the
// radial faces, tau[N_r] = 0.  One wavefront per radial column walks it from the outer
// end in chunks of 64 cells (coalesced loads and stores); inside a chunk a suffix scan
// by shuffles, across chunks a running carry, all in float64 in a fixed order.  The
// Rosseland table sits in LDS for the binary search of each cell's node, and the loads
// of kTauPre chunks are issued before either is used.  The kernel is bound by the
// float64 log and exp of the log-log interpolation: deeper prefetch (4, 8 chunks) only
// costs registers (0.70 / 0.71 / 0.76 ms at 512x256x512 for 2 / 4 / 8).
constexpr int kTauPre = 2;

__global__ __launch_bounds__(kTB) void k_tau_rosseland(Dims d, Opac op, const double *__restrict__ rf,
                                                       const double *__restrict__ rho, const double *__restrict__ T,
                                                       double *__restrict__ tau)
{
    __shared__ double sT[kMaxT], slnT[kMaxT], sY[kMaxT], slnY[kMaxT];
    for (int t = threadIdx.x; t < op.nT; t += kTB) {
        sT[t] = op.T[t];
        slnT[t] = op.lnT[t];
        sY[t] = op.kR[t];
        slnY[t] = op.lnR[t];
    }
    __syncthreads();
    const long col = (long)blockIdx.x * (kTB / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (col >= (long)d.nt * d.np) return;  // whole wavefronts leave together; no barrier below
    const long c0 = col * d.nr, f0 = col * (d.nr + 1);
    if (lane == 0) tau[f0 + d.nr] = 0.0;
    double carry = 0.0;
    for (int e0 = d.nr; e0 > 0; e0 -= 64 * kTauPre) {
        // chunk q of the group covers cells [max(e - 64, 0), e) with e = e0 - 64 q
        double tv[kTauPre], rv[kTauPre], dv[kTauPre];
#pragma unroll
        for (int q = 0; q < kTauPre; q++) {
            const int e = e0 - 64 * q, s = e - 64 > 0 ? e - 64 : 0, i = s + lane;
            const bool in = e > 0 && i < e;
            const int ic = in ? i : 0;
            tv[q] = T[c0 + ic];
            rv[q] = rho[c0 + ic];
            dv[q] = rf[ic + 1] - rf[ic];
        }
#pragma unroll
        for (int q = 0; q < kTauPre; q++) {
            const int e = e0 - 64 * q, s = e - 64 > 0 ? e - 64 : 0, i = s + lane;
            if (e <= 0) break;  // uniform over the wavefront
            double v = 0.0;
            if (i < e) v = mean_opacity(sT, slnT, sY, slnY, op.nT, tv[q], nullptr) * rv[q] * dv[q];
            // suffix sum over the lanes l' >= l of this chunk
            for (int off = 1; off < 64; off <<= 1) {
                const double u = __shfl_down(v, off);
                if (lane + off < 64) v += u;
            }
            if (i < e) tau[f0 + i] = carry + v;
            carry += __shfl(v, 0);
        }
    }
}

void launch_tau_rosseland(const Dims &d, const Opac &op, const double *rf, const double *rho, const double *T,
                          double *tau, hipStream_t st)
{
    const long cols = (long)d.nt * d.np;
    const unsigned blocks = (unsigned)((cols + kTB / 64 - 1) / (kTB / 64));
    hipLaunchKernelGGL(k_tau_rosseland, dim3(blocks), dim3(kTB), 0, st, d, op, rf, rho, T, tau);
}

// E = v in every cell: the runs without diffusion keep the thermal radiation field at
// the background a T_bc^4.
__global__ __launch_bounds__(kTB) void k_fill(long n, double v, double *__restrict__ x)
{
    long c = (long)blockIdx.x * kTB + threadIdx.x;
    if (c < n) x[c] = v;
}

// Stop test of the main iteration: max_c |T_c - Told_c| / Told_c over the grid (a
// non-finite ratio counts as +inf).  Grid-stride per block, wave maxima by shuffles,
// one partial per block, and the last block to finish folds the partials; a maximum
// is exact in any order, so the result does not depend on the schedule.
__global__ __launch_bounds__(kTB) void k_max_change(long n, const double *__restrict__ T,
                                                    const double *__restrict__ Told, double *partials,
                                                    unsigned *counter, double *out)
{
    __shared__ double sh[kTB / 64];
    __shared__ int s_last;
    double m = 0.0;
    for (long c = (long)blockIdx.x * kTB + threadIdx.x; c < n; c += (long)gridDim.x * kTB) {
        double r = fabs(T[c] - Told[c]) / Told[c];
        m = r <= m ? m : (r == r ? r : INFINITY);
    }
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = sh[0];
        for (int w = 1; w < kTB / 64; w++) b = fmax(b, sh[w]);
        partials[blockIdx.x] = b;
        __threadfence();
        s_last = atomicAdd(counter, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    double t = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kTB) t = fmax(t, partials[b]);
    for (int o = 32; o > 0; o >>= 1) t = fmax(t, __shfl_xor(t, o));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kTB / 64; w++) t = fmax(t, sh[w]);
        *out = t;
        *counter = 0u;
    }
}

__global__ __launch_bounds__(kTB) void k_scale_mul(long n, const double *__restrict__ s,
                                                   const double *__restrict__ x, double *__restrict__ y)
{
    long c = (long)blockIdx.x * kTB + threadIdx.x;
    if (c < n) y[c] = s[c] * x[c];
}
__global__ __launch_bounds__(kTB) void k_scale_div(long n, const double *__restrict__ s,
                                                   const double *__restrict__ x, double *__restrict__ y)
{
    long c = (long)blockIdx.x * kTB + threadIdx.x;
    if (c < n) y[c] = x[c] / s[c];
}

static inline unsigned nb(long n) { return (unsigned)((n + kTB - 1) / kTB); }

void launch_energy(const Dims &d, const Opac &op, const double *T, const double *S, double Efloor,
                   double *E, hipStream_t st)
{
    hipLaunchKernelGGL(k_energy, dim3(nb(d.n)), dim3(kTB), 0, st, d.n, op, T, S, Efloor, E);
}

void launch_assemble(const Dims &d, const Geo &g, const Opac &op, const double *rho, const double *T,
                     const double *En, const double *q, const double *Q, double cV, double dt,
                     double Eb, double kR_bc, double *chi, double *w, double *s, double *b,
                     double *bhat, double *ahat, float *ahat32, hipStream_t st)
{
    hipLaunchKernelGGL(k_chi, dim3(nb(d.n)), dim3(kTB), 0, st, d.n, op, T, rho, chi);
    hipLaunchKernelGGL(k_asm_faces, dim3(nb(d.n)), dim3(kTB), 0, st, d, g, chi, En, rho, kR_bc, Eb, w);
    hipLaunchKernelGGL(k_asm_diag, dim3(nb(d.n)), dim3(kTB), 0, st, d, g, w, rho, T, En, q, Q, cV, dt,
                       Eb, s, b, bhat);
    hipLaunchKernelGGL(k_asm_scale, dim3(nb(d.n)), dim3(kTB), 0, st, d, w, s, ahat, ahat32);
}

void launch_newton(const Dims &d, const Opac &op, const double *E, const double *S, double *T,
                   hipStream_t st)
{
    hipLaunchKernelGGL(k_newton, dim3(nb(d.n)), dim3(kTB), 0, st, d.n, op, E, S, T);
}

void launch_force(const Dims &d, const Geo &g, const double *w, const double *chi, const double *E,
                  const double *q, double Eb, double *f, hipStream_t st)
{
    hipLaunchKernelGGL(k_force, dim3(nb(d.n)), dim3(kTB), 0, st, d, g, w, chi, E, q, Eb, f);
}

void launch_scale_mul(long n, const double *s, const double *x, double *y, hipStream_t st)
{
    hipLaunchKernelGGL(k_scale_mul, dim3(nb(n)), dim3(kTB), 0, st, n, s, x, y);
}

void launch_scale_div(long n, const double *s, const double *x, double *y, hipStream_t st)
{
    hipLaunchKernelGGL(k_scale_div, dim3(nb(n)), dim3(kTB), 0, st, n, s, x, y);
}

void launch_fill(long n, double v, double *x, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill, dim3(nb(n)), dim3(kTB), 0, st, n, v, x);
}

void launch_max_change(long n, int nblk, const double *T, const double *Told, double *partials,
                       unsigned *counter, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_max_change, dim3(nblk), dim3(kTB), 0, st, n, T, Told, partials, counter, out);
}

}  // namespace rt
