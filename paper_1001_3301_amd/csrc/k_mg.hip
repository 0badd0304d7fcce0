// Multigrid preconditioner for CG on the Jacobi-scaled FLD operator A^ (the implicit
// solve of Eq. 15).  Not part of the paper, which preconditions its Krylov solve by
// block Jacobi: a cycle whose cost per CG iteration is a few sweeps over the grid and
// whose iteration count grows slowly with the grid, where Jacobi CG's grows with the
// number of cells along a line.
//
// Levels.  A_0 = A^ (unit diagonal; couplings ar / at / ap to the +r / +theta / +phi
// neighbour, periodic in phi).  A_(l+1) = P_l^T A_l P_l with aggregates of 1 x 2 x 2
// cells: the radius is never coarsened, because on heated, optically thin grids the
// radial couplings of A^ become weak next to the angular ones and merging radial cells
// then leaves a coarse space that misses the error; a lone last row where a size is
// odd.  P_l[f, C] = B_f / Bc_C with B_0 = 1/s (the Jacobi scaling moves the unscaled
// operator's near-null vector, the constants, to 1/s) and Bc_C^2 the sum of B_f^2 over
// the aggregate, so each coarse level is again a 7-point operator, with a general
// diagonal.  Coarsening stops at one radial line, whose inverse is stored densely.
//
// Smoother.  Damped block Jacobi on phi lines: M is the diagonal and phi couplings of
// each (r, theta) line, x <- x + omega M^-1 (b - A x).  Near the poles the phi coupling
// carries almost all of a row's weight, and a point smoother would leave the error that
// is smooth along phi and rough across theta, which the coarse levels cannot represent
// either.  Each periodic line matrix is M = T + u v^T (Sherman-Morrison, gamma = -M_00):
// T tridiagonal, factored once per system; q = T^-1 u and g = T^-1 e_0 stored per line,
// so that y_0 = g . rhs is summed during the forward sweep and the correction
// y - (v.y / (1 + v.q)) q is applied during the backward sweep (two passes per sweep).
//
// Cycle.  Pre-sweep from zero, restriction of the residual, the coarse correction,
// its prolongation (inside the residual kernel of the post-sweep), post-sweep.  The
// coarse correction is the cycle one level down (V-cycle) or, on the K levels (1 to 3
// by default), two flexible-CG steps on that level preconditioned by the cycle from it
// (K-cycle): the preconditioner is then nonlinear, and the outer CG flexible.
//
// Work layout: lanes on consecutive radii, so every access of a step is one coalesced
// row segment.  The sweeps give a thread a whole (r, theta) line walking phi; the
// residual, the restriction and the K-step stencil pass a run of phi planes of a line,
// with the phi neighbours carried in registers.  The set-up runs in float64;
// the cycle stores and computes in float32 with float64 dots (the outer CG keeps
// float64 vectors, dots and the true residual).
#include <algorithm>
#include <type_traits>

#include "rt_internal.h"

namespace rt {

constexpr int kMB = 256;  // threads per block of the multigrid kernels

__device__ __forceinline__ long mg_cell(int nr, int nt, int i, int j, int k) { return i + (long)nr * (j + (long)nt * k); }

// ----------------------------------------------------------------- set-up (float64)

// 1 / s: the near-null vector of the finest level.
__global__ __launch_bounds__(kMB) void k_mg_recip(long n, const double *__restrict__ s, double *__restrict__ B)
{
    const long c = (long)blockIdx.x * kMB + threadIdx.x;
    if (c < n) B[c] = 1.0 / s[c];
}

struct MgSetLevel {
    int nt, np;
    const double *dg;  // nullptr: unit diagonal
    const double *ar, *at, *ap, *B;
};

struct MgSetOut {
    int nt, np;
    double *dg, *ar, *at, *ap, *B;
};

__device__ __forceinline__ double mg_bc(int nr, const MgSetLevel &F, int i, int J, int K)
{
    const int ft = F.nt > 1 ? 2 : 1, fp = F.np > 1 ? 2 : 1;
    double s = 0.0;
    for (int k = fp * K; k < min(fp * K + fp, F.np); k++)
        for (int j = ft * J; j < min(ft * J + ft, F.nt); j++) {
            const double b = F.B[mg_cell(nr, F.nt, i, j, k)];
            s += b * b;
        }
    return sqrt(s);
}

// One coarse cell per thread: its Galerkin row (diagonal and the three outward
// couplings), its near-null entry, and the prolongation weights w_f = B_f / Bc of its
// children.
__global__ __launch_bounds__(kMB) void k_mg_coarsen(int nr, MgSetLevel F, MgSetOut C, float *__restrict__ w)
{
    const long nc = (long)nr * C.nt * C.np;
    const long cc = (long)blockIdx.x * kMB + threadIdx.x;
    if (cc >= nc) return;
    const int i = (int)(cc % nr);
    const long rest = cc / nr;
    const int J = (int)(rest % C.nt), K = (int)(rest / C.nt);
    const int ft = F.nt > 1 ? 2 : 1, fp = F.np > 1 ? 2 : 1;
    const int j0 = ft * J, j1 = min(j0 + ft, F.nt), k0 = fp * K, k1 = min(k0 + fp, F.np);
    const double bc = mg_bc(nr, F, i, J, K);
    auto wf = [&](int j, int k) { return F.B[mg_cell(nr, F.nt, i, j, k)] / bc; };
    double dg = 0.0;
    for (int k = k0; k < k1; k++)
        for (int j = j0; j < j1; j++) {
            const long f = mg_cell(nr, F.nt, i, j, k);
            const double wv = wf(j, k);
            w[f] = (float)wv;
            dg += (F.dg ? F.dg[f] : 1.0) * wv * wv;
        }
    // internal couplings, counted twice (a_fg and a_gf)
    if (j1 - j0 == 2)
        for (int k = k0; k < k1; k++) dg += 2.0 * F.at[mg_cell(nr, F.nt, i, j0, k)] * wf(j0, k) * wf(j0 + 1, k);
    if (k1 - k0 == 2) {
        for (int j = j0; j < j1; j++) dg += 2.0 * F.ap[mg_cell(nr, F.nt, i, j, k0)] * wf(j, k0) * wf(j, k0 + 1);
        if (F.np == 2)  // the periodic coupling of two phi cells merged into one
            for (int j = j0; j < j1; j++) dg += 2.0 * F.ap[mg_cell(nr, F.nt, i, j, 1)] * wf(j, 1) * wf(j, 0);
    }
    double ar = 0.0;
    if (i + 1 < nr) {
        const double bn = mg_bc(nr, F, i + 1, J, K);
        for (int k = k0; k < k1; k++)
            for (int j = j0; j < j1; j++) {
                const long f = mg_cell(nr, F.nt, i, j, k);
                ar += F.ar[f] * wf(j, k) * (F.B[f + 1] / bn);
            }
    }
    double at = 0.0;
    if (ft == 2 && j0 + 2 < F.nt) {  // from the last child row 2J+1 to row 2J+2
        const double bn = mg_bc(nr, F, i, J + 1, K);
        for (int k = k0; k < k1; k++) {
            const long f = mg_cell(nr, F.nt, i, j0 + 1, k);
            at += F.at[f] * wf(j0 + 1, k) * (F.B[f + nr] / bn);
        }
    }
    double ap = 0.0;
    if (fp == 2 && C.np >= 2) {  // from the last child plane towards the next aggregate
        const int kl = k1 - 1, kn = (kl + 1) % F.np;
        const double bn = mg_bc(nr, F, i, J, (K + 1) % C.np);
        for (int j = j0; j < j1; j++)
            ap += F.ap[mg_cell(nr, F.nt, i, j, kl)] * wf(j, kl) * (F.B[mg_cell(nr, F.nt, i, j, kn)] / bn);
    }
    C.dg[cc] = dg;
    C.ar[cc] = ar;
    C.at[cc] = at;
    C.ap[cc] = ap;
    C.B[cc] = bc;
}

struct MgLineOut {
    float *im, *cp, *q, *g, *rho, *kap;
};

// Factors of each phi line's matrix M (one thread per (r, theta) line).  Lines of one
// cell: 1 / M_00.  Two cells: the 2 x 2 matrix, whose off-diagonal is the sum of the
// two couplings between them.  Three or more: T = M - u v^T with u = (gamma, 0, .., 0,
// e_(m-1)), v = (1, 0, .., 0, e_(m-1) / gamma), gamma = -M_00, where e_(m-1) couples the
// last cell to the first; Thomas factors 1 / m_k and c_k = e_k / m_k of T, and q = T^-1 u,
// g = T^-1 e_0, rho = e_(m-1) / gamma, kap = 1 / (1 + q_0 + rho q_(m-1)).  tm and td are
// float64 scratch of the level's size.
constexpr int kFU = 8;  // steps whose loads the set-up walks issue together

__global__ __launch_bounds__(kMB) void k_mg_line_factor(int nr, MgSetLevel L, MgLineOut o, double *__restrict__ tm,
                                                        double *__restrict__ td)
{
    const long lines = (long)nr * L.nt;
    const long line = (long)blockIdx.x * kMB + threadIdx.x;
    if (line >= lines) return;
    const long plane = lines;
    const int m = L.np;
    auto dgv = [&](long c) { return L.dg ? L.dg[c] : 1.0; };
    if (m == 1) {
        o.im[line] = (float)(1.0 / dgv(line));
        o.cp[line] = o.q[line] = o.g[line] = 0.0f;
        o.rho[line] = o.kap[line] = 0.0f;
        return;
    }
    if (m == 2) {
        const long c1 = line + plane;
        const double e = L.ap[line] + L.ap[c1];
        const double m0 = dgv(line), m1 = dgv(c1) - e * e / m0;
        o.im[line] = (float)(1.0 / m0);
        o.im[c1] = (float)(1.0 / m1);
        o.cp[line] = (float)(e / m0);
        o.cp[c1] = 0.0f;
        o.q[line] = o.q[c1] = o.g[line] = o.g[c1] = 0.0f;
        o.rho[line] = o.kap[line] = 0.0f;
        return;
    }
    const double d0 = dgv(line), gam = -d0;
    const long cl = line + (long)(m - 1) * plane;
    const double ew = L.ap[cl];  // couples the last cell to the first
    // Each pass is a sequential walk along the line; the loads of kFU consecutive steps
    // are issued together before their part of the recurrence.
    // factor T: diagonal 2 d_0, d_k, d_(m-1) - ew^2 / gamma; off-diagonals e_k = ap_k
    double mk = d0 - gam, eprev = 0.0;
    for (int k0 = 0; k0 < m; k0 += kFU) {
        double dv[kFU], av[kFU];
#pragma unroll
        for (int u = 0; u < kFU; u++) {
            const long c = line + (long)min(k0 + u, m - 1) * plane;
            dv[u] = dgv(c);
            av[u] = L.ap[c];
        }
#pragma unroll
        for (int u = 0; u < kFU; u++) {
            const int k = k0 + u;
            if (k < m) {
                const long c = line + (long)k * plane;
                if (k > 0) {
                    double t = dv[u];
                    if (k == m - 1) t -= ew * ew / gam;
                    mk = t - eprev * eprev / mk;
                }
                tm[c] = 1.0 / mk;
                o.im[c] = (float)(1.0 / mk);
                const double e = (k < m - 1) ? av[u] : 0.0;
                o.cp[c] = (float)(e / mk);
                eprev = e;
            }
        }
    }
    // two solves with T: u and e_0
    double q0 = 0.0, qm = 0.0;
    for (int s = 0; s < 2; s++) {
        double dprev = 0.0;
        eprev = 0.0;
        for (int k0 = 0; k0 < m; k0 += kFU) {
            double tv[kFU], av[kFU];
#pragma unroll
            for (int u = 0; u < kFU; u++) {
                const long c = line + (long)min(k0 + u, m - 1) * plane;
                tv[u] = tm[c];
                av[u] = L.ap[c];
            }
#pragma unroll
            for (int u = 0; u < kFU; u++) {
                const int k = k0 + u;
                if (k < m) {
                    const long c = line + (long)k * plane;
                    const double rhs = s == 0 ? (k == 0 ? gam : (k == m - 1 ? ew : 0.0)) : (k == 0 ? 1.0 : 0.0);
                    dprev = (rhs - eprev * dprev) * tv[u];
                    td[c] = dprev;
                    eprev = (k < m - 1) ? av[u] : 0.0;
                }
            }
        }
        double y = 0.0;
        for (int k0 = m - 1; k0 >= 0; k0 -= kFU) {
            double dv[kFU], tv[kFU], av[kFU];
#pragma unroll
            for (int u = 0; u < kFU; u++) {
                const long c = line + (long)max(k0 - u, 0) * plane;
                dv[u] = td[c];
                tv[u] = tm[c];
                av[u] = L.ap[c];
            }
#pragma unroll
            for (int u = 0; u < kFU; u++) {
                const int k = k0 - u;
                if (k >= 0) {
                    const long c = line + (long)k * plane;
                    const double e = (k < m - 1) ? av[u] : 0.0;
                    y = dv[u] - e * tv[u] * y;
                    if (s == 0) {
                        o.q[c] = (float)y;
                        if (k == 0) q0 = y;
                        if (k == m - 1) qm = y;
                    } else {
                        o.g[c] = (float)y;
                    }
                }
            }
        }
    }
    const double rho = ew / gam;
    o.rho[line] = (float)rho;
    o.kap[line] = (float)(1.0 / (1.0 + q0 + rho * qm));
}

// The coarsest level, one radial line (unit diagonal when dg is null): Thomas factors
// (one thread), then the columns of its inverse (one thread per column, column-major).
__global__ void k_mg_radial_factor(int nr, const double *__restrict__ dg, const double *__restrict__ ar,
                                   double *__restrict__ im, double *__restrict__ cp)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double mk = dg ? dg[0] : 1.0;
    for (int i = 0; i < nr; i++) {
        if (i > 0) mk = (dg ? dg[i] : 1.0) - ar[i - 1] * ar[i - 1] / mk;
        im[i] = 1.0 / mk;
        cp[i] = (i + 1 < nr) ? ar[i] / mk : 0.0;
    }
}

__global__ __launch_bounds__(kMB) void k_mg_radial_inverse(int nr, const double *__restrict__ ar,
                                                           const double *__restrict__ im,
                                                           const double *__restrict__ cp, double *__restrict__ inv)
{
    const int col = blockIdx.x * kMB + threadIdx.x;
    if (col >= nr) return;
    double *x = inv + (long)col * nr;
    double d = 0.0;
    for (int i = 0; i < nr; i++) {
        const double rhs = i == col ? 1.0 : 0.0;
        d = (rhs - (i > 0 ? ar[i - 1] : 0.0) * d) * im[i];
        x[i] = d;
    }
    double y = 0.0;
    for (int i = nr - 1; i >= 0; i--) {
        y = x[i] - cp[i] * y;
        x[i] = y;
    }
}

// ------------------------------------------------------------------ V-cycle (float32)

// Block sum of a float64 per-thread value (valid in thread 0).
__device__ __forceinline__ double mg_block_sum(double v, double *sh)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kMB / 64; w++) t += sh[w];
    __syncthreads();
    return t;
}

// Two float64 sums over the grid, reduced deterministically: block partials (pairs)
// summed in block order by the last block to finish, which returns true (totals valid
// in thread 0) and clears the counter for the next use.
__device__ __forceinline__ bool mg_reduce2(double a, double b, double *partials, unsigned *counter, double *ta,
                                           double *tb)
{
    __shared__ double sh[kMB / 64];
    __shared__ int s_last;
    const double ba = mg_block_sum(a, sh), bb = mg_block_sum(b, sh);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = ba;
        partials[2 * blockIdx.x + 1] = bb;
        __threadfence();
        const unsigned prev = atomicAdd(counter, 1u);
        s_last = prev == gridDim.x - 1;
    }
    __syncthreads();
    if (!s_last) return false;
    __threadfence();
    double x = 0.0, y = 0.0;
    for (int t = threadIdx.x; t < (int)gridDim.x; t += kMB) {
        x += partials[2 * t];
        y += partials[2 * t + 1];
    }
    x = mg_block_sum(x, sh);
    y = mg_block_sum(y, sh);
    if (threadIdx.x == 0) {
        *ta = x;
        *tb = y;
        *counter = 0u;
    }
    return true;
}

// The outer CG's scalars from r.z and z.q_old: rr = r.z (alpha = rr / p.q in the
// direction kernel) and the flexible-CG beta = -(z.q_old) / (p_old.q_old) (0 after a
// restart), which equals the classical r.z / r.z_prev for a fixed preconditioner and
// keeps the directions conjugate when the preconditioner varies (the K-cycle's inner
// Krylov steps make it nonlinear).
__device__ __forceinline__ void mg_finish_dot(double rz, double zq, double *partials, unsigned *counter,
                                              DevScalars *sc, int restart)
{
    double a, b;
    if (mg_reduce2(rz, zq, partials, counter, &a, &b) && threadIdx.x == 0) {
        sc->beta = (restart || !(sc->pq != 0.0)) ? 0.0 : -b / sc->pq;
        sc->rr = a;
    }
}

// One damped block-Jacobi sweep on phi lines given its right-hand side: x = xin +
// omega M^-1 rhs, where rhs = b - A xin (k_mg_resid) or, with ZERO (xin = 0), b itself
// (float64 on the finest level: the CG residual).  The sweeps along a line are
// sequential, so the loads of kMU consecutive steps are issued together before their
// part of the recurrence (a step's latency is paid once per group, not per step).  DOT
// (the last sweep of a cycle, finest level): x goes out as the float64 z, and r.z and
// the CG scalars are formed on the way.  rhs may be L.dp: each step reads its entry
// before the forward sweep overwrites it.
constexpr int kMU = 8;

template <bool ZERO, typename BT, bool DOT>
__global__ __launch_bounds__(kMB) void k_mg_line(int nr, MgLevel L, const BT *rhs, const float *__restrict__ xin,
                                                 float *__restrict__ xout, double *__restrict__ z,
                                                 const double *__restrict__ r, const double *__restrict__ qold,
                                                 float omega, double *partials, unsigned *counter, DevScalars *sc,
                                                 int restart)
{
    if (sc && sc->done) return;
    const long lines = (long)nr * L.nt;
    const long line = (long)blockIdx.x * kMB + threadIdx.x;
    const int m = L.np;
    const long plane = lines;
    double acc = 0.0, acq = 0.0;
    if (line < lines) {
        const float *__restrict__ im = L.im;
        const float *__restrict__ cp = L.cp;
        const float *__restrict__ qf = L.q;
        const float *__restrict__ gf = L.g;
        const float *__restrict__ ap = L.ap;
        float *dp = L.dp;
        const bool sm = m >= 3;  // Sherman-Morrison correction (periodic line of 3 or more)
        const float e2 = m == 2 ? ap[line] + ap[line + plane] : 0.0f;
        float d = 0.0f, eprev = 0.0f, sg = 0.0f;
        for (int k0 = 0; k0 < m; k0 += kMU) {
            float rv[kMU], imv[kMU], gv[kMU], apv[kMU];
#pragma unroll
            for (int u = 0; u < kMU; u++) {
                const int k = k0 + u;
                if (k < m) {
                    const long c = line + (long)k * plane;
                    rv[u] = (float)rhs[c];
                    imv[u] = im[c];
                    apv[u] = ap[c];
                    gv[u] = sm ? gf[c] : 0.0f;
                }
            }
#pragma unroll
            for (int u = 0; u < kMU; u++) {
                const int k = k0 + u;
                if (k < m) {
                    d = (rv[u] - eprev * d) * imv[u];
                    dp[line + (long)k * plane] = d;
                    sg = fmaf(gv[u], rv[u], sg);
                    eprev = sm ? apv[u] : e2;
                }
            }
        }
        const float fac = sm ? L.kap[line] * fmaf(L.rho[line], d, sg) : 0.0f;
        float y = 0.0f;
        for (int k0 = m - 1; k0 >= 0; k0 -= kMU) {
            float dv[kMU], cv[kMU], qv[kMU], xv[kMU];
            double rr[kMU], qo[kMU];
#pragma unroll
            for (int u = 0; u < kMU; u++) {
                const int k = k0 - u;
                if (k >= 0) {
                    const long c = line + (long)k * plane;
                    dv[u] = dp[c];
                    cv[u] = cp[c];
                    qv[u] = sm ? qf[c] : 0.0f;
                    xv[u] = ZERO ? 0.0f : xin[c];
                    rr[u] = DOT ? r[c] : 0.0;
                    qo[u] = DOT ? qold[c] : 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < kMU; u++) {
                const int k = k0 - u;
                if (k >= 0) {
                    y = dv[u] - cv[u] * y;
                    const float delta = fmaf(-fac, qv[u], y);
                    const float xn = fmaf(omega, delta, xv[u]);
                    const long c = line + (long)k * plane;
                    if (DOT) {
                        z[c] = (double)xn;
                        acc += rr[u] * (double)xn;
                        acq += qo[u] * (double)xn;
                    } else {
                        xout[c] = xn;
                    }
                }
            }
        }
    }
    if (DOT) mg_finish_dot(acc, acq, partials, counter, sc, restart);
}

// The block's place in the launch with each XCD dealt a contiguous range: consecutive
// blocks go to the eight XCDs in turn, so block id is taken as the (id / 8)-th block of
// XCD id % 8 (a bijection on [0, gridDim.x) for any grid size).
__device__ __forceinline__ unsigned mg_xcd_block()
{
    const unsigned id = blockIdx.x, nb = gridDim.x;
    const unsigned q = nb >> 3, rm = nb & 7, x = id & 7;
    return x * q + min(x, rm) + (id >> 3);
}

// rhs = b - A x' on one level, where x' = x + P xc: the coarse correction prolonged on
// the fly, at the cell and its six neighbours; x' goes to xo for the sweep that
// follows.  Each thread walks kc consecutive phi planes of one (r, theta) line,
// carrying x' and the phi coupling of the previous and current planes in registers, so
// a phi plane is read once per walk instead of three times; the loads of kRU steps are
// issued together.  Each XCD takes a contiguous range of blocks (chunk-major, line
// blocks in order), so the theta neighbours, a few blocks away, are read through the
// same L2.  The sums are formed in the order of the 7-point product (diagonal, +r, -r,
// +theta, -theta, +phi, -phi).
constexpr int kRU = 4;

template <typename BT>
__global__ __launch_bounds__(kMB) void k_mg_resid(int nr_, MgLevel F, int cnt_, int kc_, const BT *__restrict__ b,
                                                  const float *__restrict__ x, const float *__restrict__ xc,
                                                  float *__restrict__ xo, float *__restrict__ rhs,
                                                  const DevScalars *sc)
{
    if (sc && sc->done) return;
    const unsigned nr = nr_, nt = F.nt, np = F.np, cnt = cnt_, kc = kc_;
    const unsigned plane = nr * nt, nlb = (plane + kMB - 1) / kMB;
    const unsigned lid = mg_xcd_block();
    const unsigned ch = lid / nlb, line = (lid - ch * nlb) * kMB + threadIdx.x;
    if (line >= plane) return;
    const unsigned k0 = ch * kc, k1 = min(k0 + kc, np);
    const unsigned i = line % nr, j = line / nr;
    const unsigned sj = nt > 1, sk = np > 1;
    const float *__restrict__ w = F.w;
    auto xv = [&](unsigned c, unsigned ii, unsigned jj, unsigned kk) {
        return fmaf(w[c], xc[ii + nr * ((jj >> sj) + cnt * (kk >> sk))], x[c]);
    };
    // neighbours clamped to the cell itself on the boundary faces (loaded, not used)
    const unsigned ip = i + 1 < nr ? i + 1 : i, im = i > 0 ? i - 1 : i;
    const unsigned jp = j + 1 < nt ? j + 1 : j, jm = j > 0 ? j - 1 : j;
    const unsigned dip = ip - i, dim = i - im, djp = (jp - j) * nr, djm = (j - jm) * nr;
    const unsigned km0 = k0 > 0 ? k0 - 1 : np - 1;
    float xm = xv(line + plane * km0, i, j, km0);
    float apm = F.ap[line + plane * km0];
    float x0 = xv(line + plane * k0, i, j, k0);
    for (unsigned kb = k0; kb < k1; kb += kRU) {
        float xp[kRU], xrp[kRU], xrm[kRU], xtp[kRU], xtm[kRU];
        float arp[kRU], arm[kRU], atp[kRU], atm[kRU], apf[kRU], dgv[kRU], bv[kRU];
#pragma unroll
        for (int u = 0; u < kRU; u++) {
            const unsigned k = min(kb + u, k1 - 1);
            const unsigned f = line + plane * k;
            const unsigned kp = k + 1 < np ? k + 1 : 0;
            xp[u] = xv(line + plane * kp, i, j, kp);
            xrp[u] = xv(f + dip, ip, j, k);
            xrm[u] = xv(f - dim, im, j, k);
            xtp[u] = xv(f + djp, i, jp, k);
            xtm[u] = xv(f - djm, i, jm, k);
            arp[u] = F.ar[f];
            arm[u] = F.ar[f - dim];
            atp[u] = F.at[f];
            atm[u] = F.at[f - djm];
            apf[u] = F.ap[f];
            dgv[u] = F.dg ? F.dg[f] : 1.0f;
            bv[u] = (float)b[f];
        }
#pragma unroll
        for (int u = 0; u < kRU; u++) {
            const unsigned k = kb + u;
            if (k < k1) {
                const unsigned f = line + plane * k;
                float v = dgv[u] * x0;
                if (i + 1 < nr) v = fmaf(arp[u], xrp[u], v);
                if (i > 0) v = fmaf(arm[u], xrm[u], v);
                if (j + 1 < nt) v = fmaf(atp[u], xtp[u], v);
                if (j > 0) v = fmaf(atm[u], xtm[u], v);
                if (np > 1) {
                    v = fmaf(apf[u], xp[u], v);
                    v = fmaf(apm, xm, v);
                }
                rhs[f] = bv[u] - v;
                xo[f] = x0;
                xm = x0;
                x0 = xp[u];
                apm = apf[u];
            }
        }
    }
}

// The cycle's right-hand side in float32.
template <typename RT>
__global__ __launch_bounds__(kMB) void k_mg_in(long n, const RT *__restrict__ r, float *__restrict__ b,
                                               const DevScalars *sc)
{
    if (sc && sc->done) return;
    const long c = (long)blockIdx.x * kMB + threadIdx.x;
    if (c < n) b[c] = (float)r[c];
}

// bc = P^T (b - A x) on the next level: the residuals of a coarse cell's children
// weighted by w and summed phi plane by phi plane, theta row by row (b: float64 on the
// finest level, the CG residual).  Each thread walks the fine phi planes under kc
// consecutive coarse planes of one coarse (r, theta) line, its one or two child rows
// side by side, carrying x and the phi coupling of the previous and current planes in
// registers as the residual kernel does; blocks are dealt to the XCDs the same way.
template <typename BT>
__global__ __launch_bounds__(kMB) void k_mg_restrict(int nr_, MgLevel F, int cnt_, int kc_, const BT *__restrict__ b,
                                                     const float *__restrict__ x, float *__restrict__ bc,
                                                     const DevScalars *sc)
{
    if (sc && sc->done) return;
    const unsigned nr = nr_, nt = F.nt, np = F.np, cnt = cnt_, kc = kc_;
    const unsigned cplane = nr * cnt, nlb = (cplane + kMB - 1) / kMB, plane = nr * nt;
    const unsigned lid = mg_xcd_block();
    const unsigned ch = lid / nlb, cl = (lid - ch * nlb) * kMB + threadIdx.x;
    if (cl >= cplane) return;
    const unsigned i = cl % nr, J = cl / nr;
    const unsigned sk = np > 1, ft = nt > 1 ? 2 : 1;
    const unsigned j0 = ft * J, nj = (ft == 2 && j0 + 1 < nt) ? 2 : 1;
    const unsigned k0 = (ch * kc) << sk, k1 = min((ch * kc + kc) << sk, np);
    const unsigned dip = i + 1 < nr ? 1 : 0, dim = i > 0 ? 1 : 0;
    // the child rows (a lone row repeated: loaded, not used)
    unsigned jr[2], ln[2], djp[2], djm[2];
#pragma unroll
    for (int r = 0; r < 2; r++) {
        jr[r] = min(j0 + r, nt - 1);
        ln[r] = i + nr * jr[r];
        djp[r] = jr[r] + 1 < nt ? nr : 0;
        djm[r] = jr[r] > 0 ? nr : 0;
    }
    const unsigned km0 = k0 > 0 ? k0 - 1 : np - 1;
    float xm[2], apm[2], x0[2];
#pragma unroll
    for (int r = 0; r < 2; r++) {
        xm[r] = x[ln[r] + plane * km0];
        apm[r] = F.ap[ln[r] + plane * km0];
        x0[r] = x[ln[r] + plane * k0];
    }
    float acc = 0.0f;
    for (unsigned kb = k0; kb < k1; kb += kRU) {
        float xp[kRU][2], xrp[kRU][2], xrm[kRU][2], xtp[kRU][2], xtm[kRU][2];
        float arp[kRU][2], arm[kRU][2], atp[kRU][2], atm[kRU][2], apf[kRU][2], dgv[kRU][2], bv[kRU][2], wv[kRU][2];
#pragma unroll
        for (int u = 0; u < kRU; u++) {
            const unsigned k = min(kb + u, k1 - 1);
            const unsigned kp = k + 1 < np ? k + 1 : 0;
#pragma unroll
            for (int r = 0; r < 2; r++) {
                const unsigned f = ln[r] + plane * k;
                xp[u][r] = x[ln[r] + plane * kp];
                xrp[u][r] = x[f + dip];
                xrm[u][r] = x[f - dim];
                xtp[u][r] = x[f + djp[r]];
                xtm[u][r] = x[f - djm[r]];
                arp[u][r] = F.ar[f];
                arm[u][r] = F.ar[f - dim];
                atp[u][r] = F.at[f];
                atm[u][r] = F.at[f - djm[r]];
                apf[u][r] = F.ap[f];
                dgv[u][r] = F.dg ? F.dg[f] : 1.0f;
                bv[u][r] = (float)b[f];
                wv[u][r] = F.w[f];
            }
        }
#pragma unroll
        for (int u = 0; u < kRU; u++) {
            const unsigned k = kb + u;
            if (k < k1) {
#pragma unroll
                for (int r = 0; r < 2; r++) {
                    if (r < (int)nj) {
                        float v = dgv[u][r] * x0[r];
                        if (dip) v = fmaf(arp[u][r], xrp[u][r], v);
                        if (dim) v = fmaf(arm[u][r], xrm[u][r], v);
                        if (djp[r]) v = fmaf(atp[u][r], xtp[u][r], v);
                        if (djm[r]) v = fmaf(atm[u][r], xtm[u][r], v);
                        if (np > 1) {
                            v = fmaf(apf[u][r], xp[u][r], v);
                            v = fmaf(apm[r], xm[r], v);
                        }
                        acc = fmaf(wv[u][r], bv[u][r] - v, acc);
                    }
                    xm[r] = x0[r];
                    x0[r] = xp[u][r];
                    apm[r] = apf[u][r];
                }
                if (k + 1 == k1 || ((k + 1) >> sk) != (k >> sk)) {
                    bc[i + nr * (J + cnt * (k >> sk))] = acc;
                    acc = 0.0f;
                }
            }
        }
    }
}

// The coarsest level: x = A_L^-1 b by the stored inverse (symmetric; one block per row,
// the row's products summed over the block in float64).
__global__ __launch_bounds__(kMB) void k_mg_coarse(int nr, const double *__restrict__ inv, const float *__restrict__ b,
                                                   float *__restrict__ x, const DevScalars *sc)
{
    if (sc && sc->done) return;
    __shared__ double sh[kMB / 64];
    const int row = blockIdx.x;
    double acc = 0.0;
    for (int col = threadIdx.x; col < nr; col += kMB) acc += inv[(long)row * nr + col] * (double)b[col];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kMB / 64; w++) t += sh[w];
        x[row] = (float)t;
    }
}

// A grid of one radial line: z = (double) x and r.z in one block (the cycle is the
// coarsest solve alone).
__global__ __launch_bounds__(kMB) void k_mg_out_line(int nr, const float *__restrict__ x, const double *__restrict__ r,
                                                     double *__restrict__ z, DevScalars *sc, int restart)
{
    if (sc && sc->done) return;
    __shared__ double sh[kMB / 64];
    double acc = 0.0;
    for (int c = threadIdx.x; c < nr; c += kMB) {
        const double zv = (double)x[c];
        z[c] = zv;
        acc += r[c] * zv;
    }
    const double a = mg_block_sum(acc, sh);
    if (threadIdx.x == 0) {
        sc->beta = (restart || !(sc->rr > 0.0)) ? 0.0 : a / sc->rr;
        sc->rr = a;
    }
}

// ------------------------------------------------- K-cycle: flexible CG on a level

// The coarse correction of a K-cycle level is two steps of flexible CG on A_l, each
// preconditioned by the cycle from that level (Notay's K-cycle): x = a_1 p_1 + a_2 p_2
// with p_1 = z_1, p_2 = z_2 + beta p_1, beta = -(z_2.q_1) / (p_1.q_1), q = A_l p, a =
// (p.r) / (p.q), r the level's residual.  Since q_2 = A z_2 + beta q_1, one stencil pass
// over z_2 gives every product the second step needs (z.Az, z.q_1, p_1.Az, z.r, p_1.r,
// with p_1.q_1 from the first step), and the step needs no pass to form p_2 or q_2: the
// level's result is x = a_1 z_1 + a_2 (z_2 + beta z_1).  Float32 vectors, float64 dots,
// scalars on the device (ks[0] = p_1.q_1, ks[1] = a, ks[2] = beta).
constexpr int kKcBlocks = 4096;  // most blocks of the K-cycle kernels (grid-stride loops)
constexpr int kKcSums = 5;       // products reduced by the second step's stencil pass

// Block sums of N per-thread values written to partials[N * block + u] (no atomics or
// fences: the finishing kernel that reads them starts after this kernel has ended).
template <int N>
__device__ __forceinline__ void mg_block_partials(const double (&v)[N], double *partials)
{
    __shared__ double sh[kMB / 64];
#pragma unroll
    for (int u = 0; u < N; u++) {
        const double b = mg_block_sum(v[u], sh);
        if (threadIdx.x == 0) partials[N * blockIdx.x + u] = b;
    }
}

// A z on a level and the step's products, as block partials; FIRST writes q_1 = A z_1.
// The work is cut as in the residual kernel, a thread walking kc phi planes of one
// (r, theta) line with the phi neighbours in registers, and the blocks loop over these
// units (line block, chunk) when there are more than gridDim.x of them.
template <bool FIRST>
__global__ __launch_bounds__(kMB) void k_kc_az(int nr_, MgLevel F, int kc_, const float *__restrict__ z,
                                               const float *__restrict__ p1, const float *__restrict__ q1,
                                               const float *__restrict__ r, float *__restrict__ qout,
                                               double *partials, const DevScalars *sc)
{
    if (sc && sc->done) return;
    const unsigned nr = nr_, nt = F.nt, np = F.np, kc = kc_;
    const unsigned plane = nr * nt, nlb = (plane + kMB - 1) / kMB, units = nlb * ((np + kc - 1) / kc);
    double acc[kKcSums] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (unsigned uid = mg_xcd_block(); uid < units; uid += gridDim.x) {
        const unsigned ch = uid / nlb, line = (uid - ch * nlb) * kMB + threadIdx.x;
        if (line >= plane) continue;
        const unsigned k0 = ch * kc, k1 = min(k0 + kc, np);
        const unsigned i = line % nr, j = line / nr;
        const unsigned dip = i + 1 < nr ? 1 : 0, dim = i > 0 ? 1 : 0;
        const unsigned djp = j + 1 < nt ? nr : 0, djm = j > 0 ? nr : 0;
        const unsigned km0 = k0 > 0 ? k0 - 1 : np - 1;
        float zm = z[line + plane * km0], apm = F.ap[line + plane * km0], z0 = z[line + plane * k0];
        for (unsigned kb = k0; kb < k1; kb += kRU) {
            float zp[kRU], zrp[kRU], zrm[kRU], ztp[kRU], ztm[kRU];
            float arp[kRU], arm[kRU], atp[kRU], atm[kRU], apf[kRU], dgv[kRU], rv[kRU], pv[kRU], qv[kRU];
#pragma unroll
            for (int u = 0; u < kRU; u++) {
                const unsigned k = min(kb + u, k1 - 1);
                const unsigned f = line + plane * k;
                const unsigned kp = k + 1 < np ? k + 1 : 0;
                zp[u] = z[line + plane * kp];
                zrp[u] = z[f + dip];
                zrm[u] = z[f - dim];
                ztp[u] = z[f + djp];
                ztm[u] = z[f - djm];
                arp[u] = F.ar[f];
                arm[u] = F.ar[f - dim];
                atp[u] = F.at[f];
                atm[u] = F.at[f - djm];
                apf[u] = F.ap[f];
                dgv[u] = F.dg ? F.dg[f] : 1.0f;
                rv[u] = r[f];
                pv[u] = FIRST ? 0.0f : p1[f];
                qv[u] = FIRST ? 0.0f : q1[f];
            }
#pragma unroll
            for (int u = 0; u < kRU; u++) {
                const unsigned k = kb + u;
                if (k < k1) {
                    float v = dgv[u] * z0;
                    if (dip) v = fmaf(arp[u], zrp[u], v);
                    if (dim) v = fmaf(arm[u], zrm[u], v);
                    if (djp) v = fmaf(atp[u], ztp[u], v);
                    if (djm) v = fmaf(atm[u], ztm[u], v);
                    if (np > 1) {
                        v = fmaf(apf[u], zp[u], v);
                        v = fmaf(apm, zm, v);
                    }
                    const double zd = z0, vd = v, rd = rv[u];
                    acc[0] += zd * vd;
                    acc[1] += zd * rd;
                    if (FIRST) {
                        qout[line + plane * k] = v;
                    } else {
                        const double pd = pv[u];
                        acc[2] += zd * (double)qv[u];
                        acc[3] += pd * vd;
                        acc[4] += pd * rd;
                    }
                    zm = z0;
                    z0 = zp[u];
                    apm = apf[u];
                }
            }
        }
    }
    mg_block_partials<kKcSums>(acc, partials);
}

// The step's scalars from the partials of k_kc_az (one block; the blocks' partials are
// summed in block order): FIRST sets a_1, the second step beta and a_2 from its five
// products.
template <bool FIRST>
__global__ __launch_bounds__(kMB) void k_kc_fin(int nblk, const double *__restrict__ partials, double *ks,
                                                const DevScalars *sc)
{
    if (sc && sc->done) return;
    __shared__ double sh[kKcSums][kMB / 64];
    double a[kKcSums] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += kMB)
#pragma unroll
        for (int u = 0; u < kKcSums; u++) a[u] += partials[kKcSums * b + u];
    // the five block sums together (one barrier), each as mg_block_sum forms it
#pragma unroll
    for (int u = 0; u < kKcSums; u++) {
        for (int o = 32; o > 0; o >>= 1) a[u] += __shfl_xor(a[u], o);
        if ((threadIdx.x & 63) == 0) sh[u][threadIdx.x >> 6] = a[u];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[kKcSums];
#pragma unroll
        for (int u = 0; u < kKcSums; u++) {
            t[u] = 0.0;
            for (int w = 0; w < kMB / 64; w++) t[u] += sh[u][w];
        }
        if (FIRST) {  // p_1 = z_1, q_1 = A z_1
            ks[0] = t[0];
            ks[1] = t[0] != 0.0 ? t[1] / t[0] : 0.0;
        } else {
            const double pq1 = ks[0];
            const double beta = pq1 != 0.0 ? -t[2] / pq1 : 0.0;
            const double pq = t[0] + beta * (t[2] + t[3]) + beta * beta * pq1;  // p_2.q_2
            const double pr = t[1] + beta * t[4];                                // p_2.r
            ks[2] = beta;
            ks[1] = pq != 0.0 ? pr / pq : 0.0;
        }
    }
}

// FIRST: x = a_1 z_1, r -= a_1 q_1.  Second step: x += a_2 (z_2 + beta z_1).
template <bool FIRST>
__global__ __launch_bounds__(kMB) void k_kc_upd(long n_, float *__restrict__ x, const float *__restrict__ z,
                                                const float *__restrict__ p1, const float *__restrict__ q1,
                                                float *__restrict__ r, const double *ks, const DevScalars *sc)
{
    if (sc && sc->done) return;
    const unsigned n = (unsigned)n_;
    const float a = (float)ks[1], beta = (float)ks[2];
    for (unsigned f = blockIdx.x * kMB + threadIdx.x; f < n; f += gridDim.x * kMB) {
        if (FIRST) {
            x[f] = a * z[f];
            r[f] = fmaf(-a, q1[f], r[f]);
        } else {
            x[f] = fmaf(a, fmaf(beta, p1[f], z[f]), x[f]);
        }
    }
}

// ------------------------------------------------------------------ host side

static unsigned mg_blocks(long n) { return (unsigned)((n + kMB - 1) / kMB); }

// The residual's phi planes per thread: 16 on the large levels (4M cells or more, at
// least 256K threads), else kRU (one batch of loads, the latency of one cell).
static unsigned mg_resid_planes(long cells) { return cells >= (1L << 22) ? 16u : (unsigned)kRU; }

// The restriction's coarse phi planes per thread: 8 (16 fine planes) on the large
// levels, else 2 (one batch of kRU fine planes).
template <typename BT>
static void launch_mg_restrict(int nr, const MgLevel &F, const MgLevel &C, const BT *b, const float *x, float *bc,
                               const DevScalars *sc, hipStream_t st)
{
    const unsigned kc = F.n >= (1L << 22) ? 8u : 2u;
    const unsigned nb = mg_blocks((long)nr * C.nt) * (unsigned)((C.np + kc - 1) / kc);
    hipLaunchKernelGGL((k_mg_restrict<BT>), dim3(nb), dim3(kMB), 0, st, nr, F, C.nt, (int)kc, b, x, bc, sc);
}

template <typename BT>
static void launch_mg_resid(int nr, const MgLevel &F, int cnt, const BT *b, const float *x, const float *xc, float *xo,
                            float *rhs, const DevScalars *sc, hipStream_t st)
{
    const long lines = (long)nr * F.nt;
    const unsigned kc = mg_resid_planes(F.n);
    const unsigned nb = mg_blocks(lines) * (unsigned)((F.np + kc - 1) / kc);
    hipLaunchKernelGGL((k_mg_resid<BT>), dim3(nb), dim3(kMB), 0, st, nr, F, cnt, (int)kc, b, x, xc, xo, rhs, sc);
}

void mg_shapes(int nt, int np, std::vector<std::pair<int, int>> &out)
{
    out.clear();
    out.push_back({nt, np});
    while ((long)nt * np > 1) {
        nt = nt > 1 ? (nt + 1) / 2 : 1;
        np = np > 1 ? (np + 1) / 2 : 1;
        out.push_back({nt, np});
    }
}

void launch_mg_setup(MgHier &h, const double *ahat, const double *s, hipStream_t st)
{
    const int nr = h.nr;
    const int L = (int)h.lev.size() - 1;
    const long n0 = h.lev[0].n;
    hipLaunchKernelGGL(k_mg_recip, dim3(mg_blocks(n0)), dim3(kMB), 0, st, n0, s, h.B0);
    for (int l = 0; l < L; l++) {
        const MgLevel &F = h.lev[l];
        const MgLevel &Cl = h.lev[l + 1];
        MgSetLevel sf{F.nt, F.np, l == 0 ? nullptr : h.d64[l - 1].dg, l == 0 ? ahat : h.d64[l - 1].ar,
                      l == 0 ? ahat + n0 : h.d64[l - 1].at, l == 0 ? ahat + 2 * n0 : h.d64[l - 1].ap,
                      l == 0 ? h.B0 : h.d64[l - 1].B};
        MgSetOut so{Cl.nt, Cl.np, h.d64[l].dg, h.d64[l].ar, h.d64[l].at, h.d64[l].ap, h.d64[l].B};
        hipLaunchKernelGGL(k_mg_coarsen, dim3(mg_blocks(Cl.n)), dim3(kMB), 0, st, nr, sf, so, h.w[l]);
        MgLineOut lo{h.im[l], h.cp[l], h.q[l], h.g[l], h.rho[l], h.kap[l]};
        hipLaunchKernelGGL(k_mg_line_factor, dim3(mg_blocks((long)nr * F.nt)), dim3(kMB), 0, st, nr, sf, lo, h.t64a,
                           h.t64b);
        // the next level's operator in float32
        launch_d2f(Cl.n, h.d64[l].dg, h.dg32[l], st);
        launch_d2f(Cl.n, h.d64[l].ar, h.ar32[l], st);
        launch_d2f(Cl.n, h.d64[l].at, h.at32[l], st);
        launch_d2f(Cl.n, h.d64[l].ap, h.ap32[l], st);
    }
    // the coarsest line (the finest level itself when the grid is one radial line:
    // unit diagonal)
    const double *dgL = L == 0 ? nullptr : h.d64[L - 1].dg;
    const double *arL = L == 0 ? ahat : h.d64[L - 1].ar;
    hipLaunchKernelGGL(k_mg_radial_factor, dim3(1), dim3(64), 0, st, nr, dgL, arL, h.cim, h.ccp);
    hipLaunchKernelGGL(k_mg_radial_inverse, dim3(mg_blocks(nr)), dim3(kMB), 0, st, nr, arL, h.cim, h.ccp, h.inv);
}

// The cycle as launched: pre-sweep from zero, restriction, the coarse correction
// (the coarsest solve, a K-cycle step pair on the K levels, else the cycle one level
// down), the residual with the prolonged correction, post-sweep.
struct MgRun {
    MgHier &h;
    float omega;
    DevScalars *sc;
    hipStream_t st;
};

static void mg_solve_level(MgRun &R, int l, float *b, float *out);

// The cycle from level l >= 1 on b (not modified), result in out.
static void mg_cycle(MgRun &R, int l, const float *b, float *out)
{
    MgHier &h = R.h;
    const int nr = h.nr;
    MgLevel &F = h.lev[l];
    MgLevel &C = h.lev[l + 1];
    const unsigned gl = mg_blocks((long)nr * F.nt);
    hipLaunchKernelGGL((k_mg_line<true, float, false>), dim3(gl), dim3(kMB), 0, R.st, nr, F, b, (const float *)nullptr,
                       F.x, (double *)nullptr, (const double *)nullptr, (const double *)nullptr, R.omega,
                       (double *)nullptr, (unsigned *)nullptr, R.sc, 0);
    launch_mg_restrict<float>(nr, F, C, b, F.x, C.b, R.sc, R.st);
    mg_solve_level(R, l + 1, C.b, C.xr);
    launch_mg_resid<float>(nr, F, C.nt, b, F.x, C.xr, F.x2, F.dp, R.sc, R.st);
    hipLaunchKernelGGL((k_mg_line<false, float, false>), dim3(gl), dim3(kMB), 0, R.st, nr, F, (const float *)F.dp,
                       (const float *)F.x2, out, (double *)nullptr, (const double *)nullptr, (const double *)nullptr,
                       R.omega, (double *)nullptr, (unsigned *)nullptr, R.sc, 0);
}

// Two flexible-CG steps on level l with the cycle as preconditioner; b is the level's
// residual and is updated in place.  K.p1 holds z_1 (= p_1), K.q A z_1, K.z z_2.
static void mg_kcycle(MgRun &R, int l, float *b, float *out)
{
    MgHier &h = R.h;
    MgLevel &F = h.lev[l];
    const int nr = h.nr;
    MgKLevel &K = h.kl[l];
    const DevScalars *csc = R.sc;
    const unsigned gk = (unsigned)std::min<long>((F.n + 4 * kMB - 1) / (4 * kMB), kKcBlocks);  // >= 4 cells a thread
    const unsigned kc = mg_resid_planes(F.n);
    const unsigned ga = (unsigned)std::min<long>((long)mg_blocks((long)nr * F.nt) * ((F.np + kc - 1) / kc), kKcBlocks);
    mg_cycle(R, l, b, K.p1);
    hipLaunchKernelGGL(k_kc_az<true>, dim3(ga), dim3(kMB), 0, R.st, nr, F, (int)kc, (const float *)K.p1,
                       (const float *)nullptr, (const float *)nullptr, (const float *)b, K.q, h.kpart, csc);
    hipLaunchKernelGGL(k_kc_fin<true>, dim3(1), dim3(kMB), 0, R.st, (int)ga, (const double *)h.kpart, K.ks, csc);
    hipLaunchKernelGGL(k_kc_upd<true>, dim3(gk), dim3(kMB), 0, R.st, F.n, out, (const float *)K.p1,
                       (const float *)nullptr, (const float *)K.q, b, (const double *)K.ks, csc);
    mg_cycle(R, l, b, K.z);
    hipLaunchKernelGGL(k_kc_az<false>, dim3(ga), dim3(kMB), 0, R.st, nr, F, (int)kc, (const float *)K.z,
                       (const float *)K.p1, (const float *)K.q, (const float *)b, (float *)nullptr, h.kpart, csc);
    hipLaunchKernelGGL(k_kc_fin<false>, dim3(1), dim3(kMB), 0, R.st, (int)ga, (const double *)h.kpart, K.ks, csc);
    hipLaunchKernelGGL(k_kc_upd<false>, dim3(gk), dim3(kMB), 0, R.st, F.n, out, (const float *)K.z,
                       (const float *)K.p1, (const float *)nullptr, b, (const double *)K.ks, csc);
}

static void mg_solve_level(MgRun &R, int l, float *b, float *out)
{
    MgHier &h = R.h;
    const int L = (int)h.lev.size() - 1;
    if (l == L)
        hipLaunchKernelGGL(k_mg_coarse, dim3(h.nr), dim3(kMB), 0, R.st, h.nr, (const double *)h.inv, (const float *)b,
                           out, (const DevScalars *)R.sc);
    else if (l <= h.kmax && h.kl[l].z)
        mg_kcycle(R, l, b, out);
    else
        mg_cycle(R, l, b, out);
}

// The preconditioner on the outer residual r (n_0 values): z = M_mg r, either in float64
// (z64, with r.z and z.q_old formed on the way for the outer CG, see mg_finish_dot) or
// in float32 (z32).
template <typename RT>
static void mg_vcycle(MgHier &h, const RT *r, double *z64, const double *qold, float *z32, float omega,
                      DevScalars *sc, int restart, hipStream_t st)
{
    const int nr = h.nr;
    const int L = (int)h.lev.size() - 1;
    const DevScalars *csc = sc;
    MgRun R{h, omega, sc, st};
    MgLevel &F = h.lev[0];
    if (L == 0) {  // one radial line: the exact solve
        hipLaunchKernelGGL(k_mg_in<RT>, dim3(mg_blocks(F.n)), dim3(kMB), 0, st, F.n, r, F.b, csc);
        float *x = z64 ? F.x2 : z32;
        hipLaunchKernelGGL(k_mg_coarse, dim3(nr), dim3(kMB), 0, st, nr, (const double *)h.inv, (const float *)F.b, x,
                           csc);
        if constexpr (std::is_same<RT, double>::value)
            if (z64)
                hipLaunchKernelGGL(k_mg_out_line, dim3(1), dim3(kMB), 0, st, nr, (const float *)x, r, z64, sc,
                                   restart);
        return;
    }
    MgLevel &C = h.lev[1];
    const unsigned gl = mg_blocks((long)nr * F.nt);
    hipLaunchKernelGGL((k_mg_line<true, RT, false>), dim3(gl), dim3(kMB), 0, st, nr, F, r, (const float *)nullptr, F.x,
                       (double *)nullptr, (const double *)nullptr, (const double *)nullptr, omega, (double *)nullptr,
                       (unsigned *)nullptr, sc, 0);
    launch_mg_restrict<RT>(nr, F, C, r, F.x, C.b, csc, st);
    mg_solve_level(R, 1, C.b, C.xr);
    launch_mg_resid<RT>(nr, F, C.nt, r, F.x, C.xr, F.x2, F.b, csc, st);
    bool wrote = false;
    if constexpr (std::is_same<RT, double>::value)
        if (z64) {
            hipLaunchKernelGGL((k_mg_line<false, float, true>), dim3(gl), dim3(kMB), 0, st, nr, F, (const float *)F.b,
                               (const float *)F.x2, (float *)nullptr, z64, r, qold, omega, h.part, h.cnt, sc,
                               restart);
            wrote = true;
        }
    if (!wrote)
        hipLaunchKernelGGL((k_mg_line<false, float, false>), dim3(gl), dim3(kMB), 0, st, nr, F, (const float *)F.b,
                           (const float *)F.x2, z32, (double *)nullptr, (const double *)nullptr,
                           (const double *)nullptr, omega, (double *)nullptr, (unsigned *)nullptr, sc, 0);
}

void launch_mg_vcycle(MgHier &h, const double *r, double *z, const double *qold, float omega, DevScalars *sc,
                      int restart, hipStream_t st)
{
    mg_vcycle<double>(h, r, z, qold, nullptr, omega, sc, restart, st);
}

void launch_mg_vcycle32(MgHier &h, const float *r, float *z, float omega, DevScalars *sc, hipStream_t st)
{
    mg_vcycle<float>(h, r, nullptr, nullptr, z, omega, sc, 0, st);
}

}  // namespace rt
