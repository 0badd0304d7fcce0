// Matrix-free Krylov kernels on the Jacobi-scaled 7-point spherical FLD operator
// (the paper's implicit solve of Eq. 15, Sect. "The generalized minimal residual
// method"; here CG, since the scaled operator is symmetric positive definite).
//
// The operator has unit diagonal and three off-diagonal arrays (outward r, theta, phi
// faces of each cell); the inward couplings are the neighbours' outward entries.
// One CG iteration is two kernels:
//   dir : p = r + beta p_old (recomputed for the six neighbours), q = A p, dot p.q
//   upd : y += alpha p, r -= alpha q, dot r.r
// Every dot product is accumulated in float64 and reduced deterministically: a fixed
// tree inside each block, one partial per block, and the last block to finish sums
// the partials in index order and updates the scalars (alpha, beta, convergence
// flag) in device memory, so the host only polls every few iterations.  Blocks own
// contiguous cell ranges, and consecutive ranges are placed on the same XCD so that
// the +-1 plane neighbours of a range are read through that XCD's L2.
#include "rt_internal.h"

namespace rt {

constexpr int kKB = 256;

__device__ __forceinline__ long logical_block(int nblk)
{
    int b = blockIdx.x;
    return (long)(b & 7) * (nblk >> 3) + (b >> 3);
}

__device__ __forceinline__ double block_sum(double v, double *sh)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kKB / 64; i++) t += sh[i];
    __syncthreads();
    return t;  // valid in thread 0
}

// Writes this block's partial; returns true in every thread of the last block to
// finish, which then holds the grand total in *total (thread 0).
__device__ __forceinline__ bool finish_reduce(double bsum, long L, int nblk, double *partials,
                                              unsigned *counter, double *sh, double *total)
{
    __shared__ int s_last;
    if (threadIdx.x == 0) {
        partials[L] = bsum;
        __threadfence();
        unsigned prev = atomicAdd(counter, 1u);
        s_last = (prev == (unsigned)(nblk - 1));
    }
    __syncthreads();
    if (!s_last) return false;
    __threadfence();
    double a = 0.0;
    for (int t = threadIdx.x; t < nblk; t += kKB) a += partials[t];
    a = block_sum(a, sh);
    if (threadIdx.x == 0) {
        *total = a;
        *counter = 0u;
    }
    return true;
}

// Neighbour offsets of cell c = i + nr (j + nt k): 0 marks a missing neighbour.
struct Nbr {
    bool ip, im, jp, jm, kk;
    long kp, km;  // offsets to the phi neighbours (periodic)
};

__device__ __forceinline__ Nbr neighbours(long c, const Dims &d)
{
    Nbr n;
    int i = (int)(c % d.nr);
    long jk = c / d.nr;
    int j = (int)(jk % d.nt);
    int k = (int)(jk / d.nt);
    n.ip = i + 1 < d.nr;
    n.im = i > 0;
    n.jp = j + 1 < d.nt;
    n.jm = j > 0;
    n.kk = d.np > 1;
    n.kp = (k + 1 < d.np) ? d.plane : -(long)(d.np - 1) * d.plane;
    n.km = (k > 0) ? -d.plane : (long)(d.np - 1) * d.plane;
    return n;
}

template <typename V>
__device__ __forceinline__ V dir_val(const V *__restrict__ r, const V *__restrict__ p, V beta, bool first, long c)
{
    return first ? r[c] : fma(beta, p[c], r[c]);
}

// y = A x at cell c, with x given by a functor of the cell index (summation order:
// own, +r, -r, +theta, -theta, +phi, -phi).
template <typename V, typename F>
__device__ __forceinline__ V apply_at(long c, const Dims &d, const Nbr &nb, const V *__restrict__ a, F x)
{
    const V *ar = a, *at = a + d.n, *ap = a + 2 * d.n;
    V v = x(c);
    if (nb.ip) v += ar[c] * x(c + 1);
    if (nb.im) v += ar[c - 1] * x(c - 1);
    if (nb.jp) v += at[c] * x(c + d.nr);
    if (nb.jm) v += at[c - d.nr] * x(c - d.nr);
    if (nb.kk) {
        v += ap[c] * x(c + nb.kp);
        v += ap[c + nb.km] * x(c + nb.km);
    }
    return v;
}

// ------------------------------------------------------------------- kernels

// r = b - A y; rr = r.r.  Mode 1 (CG restart): also sets rr, beta = 0, done = 0.
__global__ __launch_bounds__(kKB) void k_resid(Dims d, int nblk, long chunk, const double *__restrict__ a,
                                               const double *__restrict__ b, const double *__restrict__ y,
                                               double *__restrict__ r, double *partials, unsigned *counter,
                                               DevScalars *sc, int restart)
{
    __shared__ double sh[kKB / 64];
    long L = logical_block(nblk);
    long c0 = L * chunk, c1 = c0 + chunk < d.n ? c0 + chunk : d.n;
    double acc = 0.0;
    for (long c = c0 + threadIdx.x; c < c1; c += kKB) {
        Nbr nb = neighbours(c, d);
        double v = b[c] - apply_at<double>(c, d, nb, a, [&](long e) { return y[e]; });
        r[c] = v;
        acc += v * v;
    }
    double bs = block_sum(acc, sh), tot;
    if (finish_reduce(bs, L, nblk, partials, counter, sh, &tot) && threadIdx.x == 0) {
        sc->res2 = tot;
        sc->inv_norm = tot > 0.0 ? 1.0 / sqrt(tot) : 0.0;
        if (restart) {
            sc->rr = tot;
            sc->beta = 0.0;
            sc->done = tot <= sc->thresh2 ? 1 : 0;
        }
    }
}

// Direction + operator + dot: p = r + beta p_old, q = A p, pq = p.q, alpha = rr / pq.
template <typename V>
__global__ __launch_bounds__(kKB) void k_cg_dir(Dims d, int nblk, long chunk, const V *__restrict__ a,
                                                const V *__restrict__ r, const V *__restrict__ pold,
                                                V *__restrict__ pnew, V *__restrict__ q, double *partials,
                                                unsigned *counter, DevScalars *sc)
{
    if (sc->done) return;
    __shared__ double sh[kKB / 64];
    const double beta_d = sc->beta;
    const bool first = beta_d == 0.0;
    const V beta = (V)beta_d;
    long L = logical_block(nblk);
    long c0 = L * chunk, c1 = c0 + chunk < d.n ? c0 + chunk : d.n;
    double acc = 0.0;
    for (long c = c0 + threadIdx.x; c < c1; c += kKB) {
        Nbr nb = neighbours(c, d);
        V pc = dir_val(r, pold, beta, first, c);
        V qc = apply_at<V>(c, d, nb, a, [&](long e) { return e == c ? pc : dir_val(r, pold, beta, first, e); });
        pnew[c] = pc;
        q[c] = qc;
        acc += (double)pc * (double)qc;
    }
    double bs = block_sum(acc, sh), tot;
    if (finish_reduce(bs, L, nblk, partials, counter, sh, &tot) && threadIdx.x == 0) {
        sc->pq = tot;
        sc->alpha = sc->rr / tot;
    }
}

// Update + dot: y += alpha p, r -= alpha q, rr' = r.r, beta = rr'/rr, convergence flag.
template <typename V>
__global__ __launch_bounds__(kKB) void k_cg_upd(Dims d, int nblk, long chunk, V *__restrict__ y,
                                                const V *__restrict__ p, V *__restrict__ r,
                                                const V *__restrict__ q, double *partials,
                                                unsigned *counter, DevScalars *sc)
{
    if (sc->done) return;
    __shared__ double sh[kKB / 64];
    const V alpha = (V)sc->alpha;
    long L = logical_block(nblk);
    long c0 = L * chunk, c1 = c0 + chunk < d.n ? c0 + chunk : d.n;
    double acc = 0.0;
    for (long c = c0 + threadIdx.x; c < c1; c += kKB) {
        y[c] = fma(alpha, p[c], y[c]);
        V rv = fma(-alpha, q[c], r[c]);
        r[c] = rv;
        acc += (double)rv * (double)rv;
    }
    double bs = block_sum(acc, sh), tot;
    if (finish_reduce(bs, L, nblk, partials, counter, sh, &tot) && threadIdx.x == 0) {
        double rr = sc->rr;
        sc->beta = tot / rr;
        sc->rr = tot;
        sc->iters += 1;
        if (tot <= sc->thresh2 || !(tot == tot)) sc->done = 1;
    }
}

// Mixed mode: r32 = r * inv_norm (float), x32 = 0, rr = r32.r32, beta = 0, done = 0.
__global__ __launch_bounds__(kKB) void k_cast_residual(Dims d, int nblk, long chunk,
                                                       const double *__restrict__ r,
                                                       float *__restrict__ r32, float *__restrict__ x32,
                                                       double *partials, unsigned *counter,
                                                       DevScalars *sc, double inner_tol)
{
    __shared__ double sh[kKB / 64];
    const double s = sc->inv_norm;
    long L = logical_block(nblk);
    long c0 = L * chunk, c1 = c0 + chunk < d.n ? c0 + chunk : d.n;
    double acc = 0.0;
    for (long c = c0 + threadIdx.x; c < c1; c += kKB) {
        float v = (float)(r[c] * s);
        r32[c] = v;
        x32[c] = 0.0f;
        acc += (double)v * (double)v;
    }
    double bs = block_sum(acc, sh), tot;
    if (finish_reduce(bs, L, nblk, partials, counter, sh, &tot) && threadIdx.x == 0) {
        sc->rr = tot;
        sc->beta = 0.0;
        sc->thresh2 = inner_tol * inner_tol * tot;
        sc->done = 0;
    }
}

// Mixed mode: y += ||r|| x32 (float64 refinement update).
__global__ __launch_bounds__(kKB) void k_refine(long n, const float *__restrict__ x32, const DevScalars *sc,
                                                double *__restrict__ y)
{
    long c = (long)blockIdx.x * kKB + threadIdx.x;
    if (c >= n) return;
    double nrm = sc->inv_norm > 0.0 ? 1.0 / sc->inv_norm : 0.0;
    y[c] = fma(nrm, (double)x32[c], y[c]);
}

// res2 = x.x (float64).
__global__ __launch_bounds__(kKB) void k_norm2(Dims d, int nblk, long chunk, const double *__restrict__ x,
                                               double *partials, unsigned *counter, DevScalars *sc)
{
    __shared__ double sh[kKB / 64];
    long L = logical_block(nblk);
    long c0 = L * chunk, c1 = c0 + chunk < d.n ? c0 + chunk : d.n;
    double acc = 0.0;
    for (long c = c0 + threadIdx.x; c < c1; c += kKB) acc += x[c] * x[c];
    double bs = block_sum(acc, sh), tot;
    if (finish_reduce(bs, L, nblk, partials, counter, sh, &tot) && threadIdx.x == 0) sc->res2 = tot;
}

// y = A x (float64), plain.
__global__ __launch_bounds__(kKB) void k_spmv(Dims d, const double *__restrict__ a, const double *__restrict__ x,
                                              double *__restrict__ y)
{
    long c = (long)blockIdx.x * kKB + threadIdx.x;
    if (c >= d.n) return;
    Nbr nb = neighbours(c, d);
    y[c] = apply_at<double>(c, d, nb, a, [&](long e) { return x[e]; });
}

// ------------------------------------------------------------------ launchers

void launch_spmv(const Dims &d, const double *a, const double *x, double *y, hipStream_t st)
{
    hipLaunchKernelGGL(k_spmv, dim3((unsigned)((d.n + kKB - 1) / kKB)), dim3(kKB), 0, st, d, a, x, y);
}

void launch_norm2(const Dims &d, int nblk, long chunk, const double *x, double *partials, unsigned *counter,
                  DevScalars *sc, hipStream_t st)
{
    hipLaunchKernelGGL(k_norm2, dim3(nblk), dim3(kKB), 0, st, d, nblk, chunk, x, partials, counter, sc);
}

void launch_resid(const Dims &d, int nblk, long chunk, const double *a, const double *b, const double *y,
                  double *r, double *partials, unsigned *counter, DevScalars *sc, int restart, hipStream_t st)
{
    hipLaunchKernelGGL(k_resid, dim3(nblk), dim3(kKB), 0, st, d, nblk, chunk, a, b, y, r, partials, counter,
                       sc, restart);
}

void launch_cg_iter64(const Dims &d, int nblk, long chunk, const double *a, double *y, double *r,
                      double *pold, double *pnew, double *q, double *partials, unsigned *counter,
                      DevScalars *sc, hipStream_t st, const hipEvent_t *ev)
{
    if (ev) (void)hipEventRecord(ev[0], st);
    hipLaunchKernelGGL(k_cg_dir<double>, dim3(nblk), dim3(kKB), 0, st, d, nblk, chunk, a, r, pold, pnew, q,
                       partials, counter, sc);
    if (ev) (void)hipEventRecord(ev[1], st);
    hipLaunchKernelGGL(k_cg_upd<double>, dim3(nblk), dim3(kKB), 0, st, d, nblk, chunk, y, pnew, r, q,
                       partials, counter, sc);
    if (ev) (void)hipEventRecord(ev[2], st);
}

void launch_cg_iter32(const Dims &d, int nblk, long chunk, const float *a, float *x, float *r, float *pold,
                      float *pnew, float *q, double *partials, unsigned *counter, DevScalars *sc,
                      hipStream_t st, const hipEvent_t *ev)
{
    if (ev) (void)hipEventRecord(ev[0], st);
    hipLaunchKernelGGL(k_cg_dir<float>, dim3(nblk), dim3(kKB), 0, st, d, nblk, chunk, a, r, pold, pnew, q,
                       partials, counter, sc);
    if (ev) (void)hipEventRecord(ev[1], st);
    hipLaunchKernelGGL(k_cg_upd<float>, dim3(nblk), dim3(kKB), 0, st, d, nblk, chunk, x, pnew, r, q,
                       partials, counter, sc);
    if (ev) (void)hipEventRecord(ev[2], st);
}

void launch_cast_residual(const Dims &d, int nblk, long chunk, const double *r, float *r32, float *x32,
                          double *partials, unsigned *counter, DevScalars *sc, double inner_tol, hipStream_t st)
{
    hipLaunchKernelGGL(k_cast_residual, dim3(nblk), dim3(kKB), 0, st, d, nblk, chunk, r, r32, x32, partials,
                       counter, sc, inner_tol);
}

void launch_refine(long n, const float *x32, const DevScalars *sc, double *y, hipStream_t st)
{
    hipLaunchKernelGGL(k_refine, dim3((unsigned)((n + kKB - 1) / kKB)), dim3(kKB), 0, st, n, x32, sc, y);
}


}  // namespace rt
