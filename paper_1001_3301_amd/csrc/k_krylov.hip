// Matrix-free Krylov kernels on the Jacobi-scaled 7-point spherical FLD operator
// (the paper's implicit solve of Eq. 15, Sect. "The generalized minimal residual
// method"; here CG, since the scaled operator is symmetric positive definite).
//
// The operator has unit diagonal and three off-diagonal arrays (outward r, theta, phi
// faces of each cell); the inward couplings are the neighbours' outward entries.
// One CG iteration is two kernels:
//   dir : p = r + beta p_old (recomputed for the six neighbours), q = A p, dot p.q
//   upd : y += alpha p, r -= alpha q, dot r.r
// Work layout: the unit of work is a radial row (one (theta, phi) column of N_r cells,
// contiguous in memory); a thread owns VW consecutive cells of a row and moves them
// with 16-byte vector loads (VW = 2 doubles or 4 floats; 1 when N_r is not a multiple
// of VW).  Each XCD owns a theta-band of rows over all phi-planes and sweeps it in
// windows (see for_segments), so the stencil's +-theta and +-phi neighbour rows are
// re-read from that XCD's L2 instead of HBM.  Row index arithmetic is incremental, so
// no division happens per cell.
// Every dot product is accumulated in float64 and reduced deterministically: a fixed
// tree inside each block, one partial per block, and the last block to finish sums
// the partials in index order and updates the scalars (alpha, beta, convergence
// flag) in device memory, so the host only polls every few iterations.
#include <cstdlib>

#include "rt_internal.h"

namespace rt {

#ifndef RTMI_KRYLOV_BLOCK
#define RTMI_KRYLOV_BLOCK 256
#endif
constexpr int kKB = RTMI_KRYLOV_BLOCK;  // threads per block of the Krylov kernels

// Index of this block's partial sum (any fixed one-to-one map works).
__device__ __forceinline__ long logical_block(int nblk)
{
    (void)nblk;
    return blockIdx.x;
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

// ------------------------------------------------------------ vector access

template <typename V, int VW>
__device__ __forceinline__ void vload(const V *__restrict__ p, V (&o)[VW])
{
    if constexpr (VW == 1) {
        o[0] = p[0];
    } else {
        struct alignas(sizeof(V) * VW) B { V v[VW]; };
        B b = *reinterpret_cast<const B *>(p);
#pragma unroll
        for (int m = 0; m < VW; m++) o[m] = b.v[m];
    }
}

template <typename V, int VW>
__device__ __forceinline__ void vstore(V *__restrict__ p, const V (&o)[VW])
{
    if constexpr (VW == 1) {
        p[0] = o[0];
    } else {
        struct alignas(sizeof(V) * VW) B { V v[VW]; };
        B b;
#pragma unroll
        for (int m = 0; m < VW; m++) b.v[m] = o[m];
        *reinterpret_cast<B *>(p) = b;
    }
}

// Non-temporal forms (the `nt` cache policy): the lines they touch are not kept for
// reuse, so a pure streaming pass does not push out of the Infinity Cache what the pass
// after it will read.
template <typename V, int VW>
__device__ __forceinline__ void vload_nt(const V *__restrict__ p, V (&o)[VW])
{
    if constexpr (VW == 1) {
        o[0] = __builtin_nontemporal_load(p);
    } else {
        typedef V T __attribute__((ext_vector_type(VW)));
        const T b = __builtin_nontemporal_load(reinterpret_cast<const T *>(p));
#pragma unroll
        for (int m = 0; m < VW; m++) o[m] = b[m];
    }
}

template <typename V, int VW>
__device__ __forceinline__ void vstore_nt(V *__restrict__ p, const V (&o)[VW])
{
    if constexpr (VW == 1) {
        __builtin_nontemporal_store(o[0], p);
    } else {
        typedef V T __attribute__((ext_vector_type(VW)));
        T b;
#pragma unroll
        for (int m = 0; m < VW; m++) b[m] = o[m];
        __builtin_nontemporal_store(b, reinterpret_cast<T *>(p));
    }
}

// A row of the grid as seen from a block: its first cell and its neighbour rows.
struct Row {
    long base;      // index of cell (0, j, k)
    bool jp, jm;    // theta neighbours exist
    bool kk;        // phi neighbours exist (N_phi > 1)
    long kp, km;    // offsets of the phi neighbours (periodic)
    int par;        // (j + k) & 1 (the colouring of the red-black kernels)
};

// Calls f(row, i) for every VW-cell segment (cells i .. i+VW-1 of a row) owned by the
// block.  The hardware deals blocks round-robin over the 8 XCDs; the rows are split
// the same way, into 8 theta-bands (all phi-planes of a band of ceil(N_theta/8) polar
// rows), one per XCD, so a row's +-theta and +-phi neighbour rows are streamed by the
// same XCD and stay in its L2.  Inside its band an XCD sweeps the rows (theta fastest,
// then phi) in windows: in round t its nloc blocks take the window of rows
// [t S, (t+1) S), S = nloc * rsub, local block l the rows [t S + l rsub, ...), so the
// +-1 plane of a row lies at most a window or two away.  The rows of a block do not
// depend on timing, which keeps the reductions deterministic.  Requires N_r % VW == 0.
template <int VW, typename F>
__device__ __forceinline__ void for_segments(const Dims &d, int nblk, F &&f)
{
    const int tpr = d.nr / VW;  // segments per row
    int sub, rsub, i0, istep;
    if (tpr >= kKB) {
        sub = 0;
        rsub = 1;
        i0 = threadIdx.x * VW;
        istep = kKB * VW;
    } else {
        rsub = kKB / tpr;
        sub = threadIdx.x / tpr;
        i0 = (threadIdx.x - sub * tpr) * VW;
        istep = d.nr;
        if (sub >= rsub) return;
    }
    const int xcd = blockIdx.x & 7, nloc = nblk >> 3, l = blockIdx.x >> 3;
    const int band = (d.nt + 7) >> 3;
    const int j0 = xcd * band;
    const int blen = d.nt - j0 < band ? d.nt - j0 : band;  // rows of this XCD's band
    if (blen <= 0) return;
    const long nrows = (long)blen * d.np;
    const long S = (long)nloc * rsub;
    long u = (long)l * rsub + sub;
    if (u >= nrows) return;
    int jb = (int)(u % blen), k = (int)(u / blen);
    const int dj = (int)(S % blen), dk = (int)(S / blen);
    const long pl = d.plane, wrap = (long)(d.np - 1) * d.plane;
    for (; u < nrows; u += S) {
        // d.rev mirrors the band (row u -> nrows - 1 - u): consecutive passes that sweep
        // in opposite directions start on the rows the previous pass touched last
        const int j = j0 + (d.rev ? blen - 1 - jb : jb), kq = d.rev ? d.np - 1 - k : k;
        Row rw;
        rw.base = ((long)kq * d.nt + j) * d.nr;
        rw.jp = j + 1 < d.nt;
        rw.jm = j > 0;
        rw.kk = d.np > 1;
        rw.kp = (kq + 1 < d.np) ? pl : -wrap;
        rw.km = (kq > 0) ? -pl : wrap;
        rw.par = (j + kq) & 1;
        for (int i = i0; i < d.nr; i += istep) f(rw, i);
        jb += dj;
        k += dk;
        if (jb >= blen) { jb -= blen; k++; }
    }
}

// p = r + beta p_old for VW cells at c (beta = 0 after a restart: fma(0, p, r) = r
// exactly, the p buffers are zeroed at creation and always finite afterwards).
template <typename V, int VW>
__device__ __forceinline__ void dir_seg(const V *__restrict__ r, const V *__restrict__ p, V beta, long c,
                                        V (&o)[VW])
{
    V t[VW];
    vload<V, VW>(r + c, o);
    vload<V, VW>(p + c, t);
#pragma unroll
    for (int m = 0; m < VW; m++) o[m] = fma(beta, t[m], o[m]);
}

template <typename V>
__device__ __forceinline__ V dir_one(const V *__restrict__ r, const V *__restrict__ p, V beta, long c)
{
    return fma(beta, p[c], r[c]);
}

// Neighbour addresses of the segment at row position i, clamped to the segment itself
// where a neighbour does not exist, and masks for the inward coefficients.  Every load
// of the stencil is unconditional (no branch splits them into serialised groups); the
// outward coefficients of boundary faces are exact zeros in the assembled operator, and
// the inward ones are masked here, so the missing terms add exactly zero.
struct Nb {
    long c, cl, cr, cjp, cjm, ckp, ckm;
    bool ml, mjm;  // inward radial / inward polar coefficient present
};

template <int VW>
__device__ __forceinline__ Nb neighbours(const Dims &d, const Row &rw, int i)
{
    Nb n;
    n.c = rw.base + i;
    n.ml = i > 0;
    n.cl = n.ml ? n.c - 1 : n.c;
    n.cr = (i + VW < d.nr) ? n.c + VW : n.c + VW - 1;
    n.cjp = rw.jp ? n.c + d.nr : n.c;
    n.mjm = rw.jm;
    n.cjm = rw.jm ? n.c - d.nr : n.c;
    n.ckp = n.c + rw.kp;  // offsets are 0 when N_phi = 1 (the phi coefficients are 0 then)
    n.ckm = n.c + rw.km;
    return n;
}

// q = A x for the VW cells of a segment: xv its values, xl / xr the radial neighbours
// and load(e, o) a loader of neighbour segments (summation order: own, +r, -r, +theta,
// -theta, +phi, -phi).
template <typename V, int VW, typename LoadSeg>
__device__ __forceinline__ void apply_seg(const Dims &d, const Nb &nb, const V *__restrict__ a, const V (&xv)[VW],
                                          V xl, V xr, LoadSeg &&load, V (&q)[VW])
{
    const V *ar = a, *at = a + d.n, *ap = a + 2 * d.n;
    V arv[VW], atp[VW], atm[VW], app[VW], apm[VW], xjp[VW], xjm[VW], xkp[VW], xkm[VW];
    vload<V, VW>(ar + nb.c, arv);
    V arl = ar[nb.cl] * (V)nb.ml;
    vload<V, VW>(at + nb.c, atp);
    vload<V, VW>(at + nb.cjm, atm);
    vload<V, VW>(ap + nb.c, app);
    vload<V, VW>(ap + nb.ckm, apm);
    load(nb.cjp, xjp);
    load(nb.cjm, xjm);
    load(nb.ckp, xkp);
    load(nb.ckm, xkm);
    const V mjm = (V)nb.mjm;
#pragma unroll
    for (int m = 0; m < VW; m++) {
        V v = xv[m];
        v += arv[m] * (m + 1 < VW ? xv[m + 1] : xr);
        v += (m > 0 ? arv[m - 1] : arl) * (m > 0 ? xv[m - 1] : xl);
        v += atp[m] * xjp[m];
        v += (atm[m] * mjm) * xjm[m];
        v += app[m] * xkp[m];
        v += apm[m] * xkm[m];
        q[m] = v;
    }
}

// ------------------------------------------------------------------- kernels

// r = b - A y; res2 = r.r.  restart = 1 (CG restart): also rr = res2, beta = 0 and
// done = (res2 <= thresh2).
template <int VW>
__device__ __forceinline__ void k_resid_body(Dims d, int nblk, const double *__restrict__ a,
                                               const double *__restrict__ b, const double *__restrict__ y,
                                               double *__restrict__ r, double *partials, unsigned *counter,
                                               DevScalars *sc, int restart)
{
    __shared__ double sh[kKB / 64];
    const long L = logical_block(nblk);
    double acc = 0.0;
    for_segments<VW>(d, nblk, [&](const Row &rw, int i) {
        const Nb nb = neighbours<VW>(d, rw, i);
        const long c = nb.c;
        double xv[VW], q[VW], bv[VW];
        vload<double, VW>(y + c, xv);
        double xl = y[nb.cl], xr = y[nb.cr];
        apply_seg<double, VW>(d, nb, a, xv, xl, xr, [&](long e, double(&o)[VW]) { vload<double, VW>(y + e, o); },
                              q);
        vload<double, VW>(b + c, bv);
#pragma unroll
        for (int m = 0; m < VW; m++) {
            q[m] = bv[m] - q[m];
            acc += q[m] * q[m];
        }
        vstore<double, VW>(r + c, q);
    });
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
template <typename V, int VW>
__global__ __launch_bounds__(kKB) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_cg_dir(Dims d, int nblk, const V *__restrict__ a,
                                                const V *__restrict__ r, const V *__restrict__ pold,
                                                V *__restrict__ pnew, V *__restrict__ q, double *partials,
                                                unsigned *counter, DevScalars *sc)
{
    if (sc->done) return;
    __shared__ double sh[kKB / 64];
    const V beta = (V)sc->beta;
    const long L = logical_block(nblk);
    double acc = 0.0;
    for_segments<VW>(d, nblk, [&](const Row &rw, int i) {
        const Nb nb = neighbours<VW>(d, rw, i);
        const long c = nb.c;
        V pv[VW], qv[VW];
        dir_seg<V, VW>(r, pold, beta, c, pv);
        V pl = dir_one(r, pold, beta, nb.cl), pr = dir_one(r, pold, beta, nb.cr);
        apply_seg<V, VW>(d, nb, a, pv, pl, pr, [&](long e, V(&o)[VW]) { dir_seg<V, VW>(r, pold, beta, e, o); },
                         qv);
        vstore<V, VW>(pnew + c, pv);
        vstore<V, VW>(q + c, qv);
#pragma unroll
        for (int m = 0; m < VW; m++) acc += (double)pv[m] * (double)qv[m];
    });
    double bs = block_sum(acc, sh), tot;
    if (finish_reduce(bs, L, nblk, partials, counter, sh, &tot) && threadIdx.x == 0) {
        sc->pq = tot;
        sc->alpha = sc->rr / tot;
    }
}

// Update + dot: y += alpha p, r -= alpha q, rr' = r.r, beta = rr'/rr, convergence flag.
// NT: all six streams with the non-temporal policy (the update of the reduced system,
// whose arrays the next pass does not read first).
template <typename V, int VW, bool NT>
__device__ __forceinline__ void cg_upd_body(Dims d, int nblk, V *__restrict__ y, const V *__restrict__ p,
                                            V *__restrict__ r, const V *__restrict__ q, double *partials,
                                            unsigned *counter, DevScalars *sc)
{
    if (sc->done) return;
    __shared__ double sh[kKB / 64];
    const V alpha = (V)sc->alpha;
    const long L = logical_block(nblk);
    double acc = 0.0;
    for_segments<VW>(d, nblk, [&](const Row &rw, int i) {
        const long c = rw.base + i;
        V yv[VW], pv[VW], rv[VW], qv[VW];
        if constexpr (NT) {
            vload_nt<V, VW>(y + c, yv);
            vload_nt<V, VW>(p + c, pv);
            vload_nt<V, VW>(r + c, rv);
            vload_nt<V, VW>(q + c, qv);
        } else {
            vload<V, VW>(y + c, yv);
            vload<V, VW>(p + c, pv);
            vload<V, VW>(r + c, rv);
            vload<V, VW>(q + c, qv);
        }
#pragma unroll
        for (int m = 0; m < VW; m++) {
            yv[m] = fma(alpha, pv[m], yv[m]);
            rv[m] = fma(-alpha, qv[m], rv[m]);
            acc += (double)rv[m] * (double)rv[m];
        }
        if constexpr (NT) {
            vstore_nt<V, VW>(y + c, yv);
            vstore_nt<V, VW>(r + c, rv);
        } else {
            vstore<V, VW>(y + c, yv);
            vstore<V, VW>(r + c, rv);
        }
    });
    double bs = block_sum(acc, sh), tot;
    if (finish_reduce(bs, L, nblk, partials, counter, sh, &tot) && threadIdx.x == 0) {
        double rr = sc->rr;
        sc->beta = tot / rr;
        sc->rr = tot;
        sc->iters += 1;
        if (tot <= sc->thresh2 || !(tot == tot)) sc->done = 1;
    }
}

template <typename V, int VW>
__global__ __launch_bounds__(kKB) void k_cg_upd(Dims d, int nblk, V *__restrict__ y, const V *__restrict__ p,
                                                V *__restrict__ r, const V *__restrict__ q, double *partials,
                                                unsigned *counter, DevScalars *sc)
{
    cg_upd_body<V, VW, false>(d, nblk, y, p, r, q, partials, counter, sc);
}

template <typename V, int VW>
__global__ __launch_bounds__(kKB) void k_cg_upd_nt(Dims d, int nblk, V *__restrict__ y, const V *__restrict__ p,
                                                   V *__restrict__ r, const V *__restrict__ q, double *partials,
                                                   unsigned *counter, DevScalars *sc)
{
    cg_upd_body<V, VW, true>(d, nblk, y, p, r, q, partials, counter, sc);
}

// Mixed mode, reliable update: r32 = float(r) from the float64 residual r = b - A y
// just computed by k_resid (after y absorbed x32), x32 = 0, rr = r32.r32, and beta
// rescaled so the next direction continues from the replaced residual
// (beta = rr_true / rr_prev); restart = 1 starts a fresh direction (beta = 0).  The
// direction is also restarted when the true residual exceeds the recurrence residual
// by more than a factor 2 in norm: the float32 recurrence then ran past the accuracy
// float32 can reach (on a system of one or a few unknowns it reaches zero within a
// chunk), the old direction says nothing about the replaced residual, and continuing
// it sends the iteration off course.  On large systems the two residuals agree to a
// few per cent at each update.
__global__ __launch_bounds__(kKB) void k_reliable(Dims d, int nblk, const double *__restrict__ r,
                                                  float *__restrict__ r32, float *__restrict__ x32,
                                                  double *__restrict__ partials, unsigned *counter,
                                                  DevScalars *sc, int restart)
{
    __shared__ double sh[kKB / 64];
    const long L = logical_block(nblk);
    double acc = 0.0;
    for_segments<1>(d, nblk, [&](const Row &rw, int i) {
        const long c = rw.base + i;
        float v = (float)r[c];
        r32[c] = v;
        x32[c] = 0.0f;
        acc += (double)v * (double)v;
    });
    double bs = block_sum(acc, sh), tot;
    if (finish_reduce(bs, L, nblk, partials, counter, sh, &tot) && threadIdx.x == 0) {
        double rr_prev = (sc->beta > 0.0) ? sc->rr / sc->beta : 0.0;
        const bool off = !(tot <= 4.0 * sc->rr);
        sc->beta = (restart || rr_prev == 0.0 || off) ? 0.0 : tot / rr_prev;
        sc->rr = tot;
        sc->done = tot <= sc->thresh2 ? 1 : 0;
    }
}

// Like finish_reduce for two sums at once (partials hold pairs).
__device__ __forceinline__ bool finish_reduce2(double a, double b, long L, int nblk, double *partials,
                                               unsigned *counter, double *sh, double *ta, double *tb)
{
    __shared__ int s_last;
    double ba = block_sum(a, sh), bb = block_sum(b, sh);
    if (threadIdx.x == 0) {
        partials[2 * L] = ba;
        partials[2 * L + 1] = bb;
        __threadfence();
        unsigned prev = atomicAdd(counter, 1u);
        s_last = (prev == (unsigned)(nblk - 1));
    }
    __syncthreads();
    if (!s_last) return false;
    __threadfence();
    double x = 0.0, y = 0.0;
    for (int t = threadIdx.x; t < nblk; t += kKB) {
        x += partials[2 * t];
        y += partials[2 * t + 1];
    }
    x = block_sum(x, sh);
    y = block_sum(y, sh);
    if (threadIdx.x == 0) {
        *ta = x;
        *tb = y;
        *counter = 0u;
    }
    return true;
}

// Flexible CG (one A-orthogonalisation), float32 vectors, float64 dots:
// p = z + beta p_old (recomputed at the neighbours), q = A p, pq = p.q, pr = p.r,
// alpha = pr / pq.
template <int VW>
__global__ __launch_bounds__(kKB) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_fcg_dir(
    Dims d, int nblk, const float *__restrict__ a, const float *__restrict__ z, const float *__restrict__ pold,
    const float *__restrict__ r, float *__restrict__ pnew, float *__restrict__ q, double *partials, unsigned *counter,
    DevScalars *sc)
{
    if (sc->done) return;
    __shared__ double sh[kKB / 64];
    const float beta = (float)sc->beta;
    const long L = logical_block(nblk);
    double acc = 0.0, acr = 0.0;
    for_segments<VW>(d, nblk, [&](const Row &rw, int i) {
        const Nb nb = neighbours<VW>(d, rw, i);
        const long c = nb.c;
        float pv[VW], qv[VW], rv[VW];
        dir_seg<float, VW>(z, pold, beta, c, pv);
        float pl = dir_one(z, pold, beta, nb.cl), pr = dir_one(z, pold, beta, nb.cr);
        apply_seg<float, VW>(d, nb, a, pv, pl, pr, [&](long e, float(&o)[VW]) { dir_seg<float, VW>(z, pold, beta, e, o); },
                             qv);
        vstore<float, VW>(pnew + c, pv);
        vstore<float, VW>(q + c, qv);
        vload<float, VW>(r + c, rv);
#pragma unroll
        for (int m = 0; m < VW; m++) {
            acc += (double)pv[m] * (double)qv[m];
            acr += (double)pv[m] * (double)rv[m];
        }
    });
    double pq, prr;
    if (finish_reduce2(acc, acr, L, nblk, partials, counter, sh, &pq, &prr) && threadIdx.x == 0) {
        sc->pq = pq;
        sc->alpha = prr / pq;
    }
}

// beta = -(z.q) / (p.q) for the next flexible-CG direction.
__global__ __launch_bounds__(kKB) void k_fcg_beta(Dims d, int nblk, const float *__restrict__ z,
                                                  const float *__restrict__ q, double *partials, unsigned *counter,
                                                  DevScalars *sc)
{
    if (sc->done) return;
    __shared__ double sh[kKB / 64];
    const long L = logical_block(nblk);
    double acc = 0.0;
    for_segments<1>(d, nblk, [&](const Row &rw, int i) {
        const long c = rw.base + i;
        acc += (double)z[c] * (double)q[c];
    });
    double bs = block_sum(acc, sh), tot;
    if (finish_reduce(bs, L, nblk, partials, counter, sh, &tot) && threadIdx.x == 0) sc->beta = -tot / sc->pq;
}

// scale = sqrt(n / rr) (the residual scaled to unit RMS enters the network), and its
// inverse; both as float64 device scalars.
__global__ void k_rms_scale(long n, const DevScalars *sc, double *scale)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double rr = sc->rr;
        double s = rr > 0.0 ? sqrt((double)n / rr) : 1.0;
        scale[0] = s;
        scale[1] = 1.0 / s;
    }
}

// y += x32 (float64 accumulation of the float32 partial solution).
__global__ __launch_bounds__(kKB) void k_fold(long n, const float *__restrict__ x32, double *__restrict__ y)
{
    long c = (long)blockIdx.x * kKB + threadIdx.x;
    if (c < n) y[c] += (double)x32[c];
}

// res2 = x.x (float64).
__global__ __launch_bounds__(kKB) void k_norm2(Dims d, int nblk, const double *__restrict__ x,
                                               double *partials, unsigned *counter, DevScalars *sc)
{
    __shared__ double sh[kKB / 64];
    const long L = logical_block(nblk);
    double acc = 0.0;
    for_segments<1>(d, nblk, [&](const Row &rw, int i) {
        double v = x[rw.base + i];
        acc += v * v;
    });
    double bs = block_sum(acc, sh), tot;
    if (finish_reduce(bs, L, nblk, partials, counter, sh, &tot) && threadIdx.x == 0) sc->res2 = tot;
}

// rr = x.x for a float32 vector (float64 accumulation): the input scale of a standalone
// application of the learned preconditioner.
__global__ __launch_bounds__(kKB) void k_norm2_rr32(Dims d, int nblk, const float *__restrict__ x,
                                                    double *partials, unsigned *counter, DevScalars *sc)
{
    __shared__ double sh[kKB / 64];
    const long L = logical_block(nblk);
    double acc = 0.0;
    for_segments<1>(d, nblk, [&](const Row &rw, int i) {
        const double v = x[rw.base + i];
        acc += v * v;
    });
    double bs = block_sum(acc, sh), tot;
    if (finish_reduce(bs, L, nblk, partials, counter, sh, &tot) && threadIdx.x == 0) sc->rr = tot;
}

// ------------------------------------------------------------------ launchers

// Bytes per array that one thread moves per segment (16, 32 or 64: one, two or four
// 16-byte loads in flight per array); more bytes in flight per wave is what a
// streaming kernel at full occupancy needs to cover HBM latency.
static int seg_bytes()
{
    static int v = [] {
        const char *e = std::getenv("RTMI_SEG_BYTES");
        int b = e ? std::atoi(e) : 16;
        return (b == 16 || b == 32 || b == 64) ? b : 16;
    }();
    return v;
}

// Largest segment width (cells) of at most `bytes` that divides N_r.
template <typename V>
static int pick_vw(const Dims &d)
{
    int vw = seg_bytes() / (int)sizeof(V);
    while (vw > 1 && d.nr % vw != 0) vw /= 2;
    return vw;
}

#define RT_DISPATCH_VW(V, vw, KERNEL, ...)                                                                \
    do {                                                                                                \
        switch (vw) {                                                                                   \
        case 16: if constexpr (sizeof(V) == 4) { hipLaunchKernelGGL((KERNEL<V, 16>), __VA_ARGS__); break; } [[fallthrough]]; \
        case 8: hipLaunchKernelGGL((KERNEL<V, 8>), __VA_ARGS__); break;                                 \
        case 4: hipLaunchKernelGGL((KERNEL<V, 4>), __VA_ARGS__); break;                                 \
        case 2: hipLaunchKernelGGL((KERNEL<V, 2>), __VA_ARGS__); break;                                 \
        default: hipLaunchKernelGGL((KERNEL<V, 1>), __VA_ARGS__); break;                                \
        }                                                                                               \
    } while (0)

template <typename V, int VW>
__global__ __launch_bounds__(kKB) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_spmv_t(Dims d, int nblk, const V *__restrict__ a, const V *__restrict__ x,
                                                V *__restrict__ y)
{
    for_segments<VW>(d, nblk, [&](const Row &rw, int i) {
        const Nb nb = neighbours<VW>(d, rw, i);
        const long c = nb.c;
        V xv[VW], q[VW];
        vload<V, VW>(x + c, xv);
        V xl = x[nb.cl], xr = x[nb.cr];
        apply_seg<V, VW>(d, nb, a, xv, xl, xr, [&](long e, V(&o)[VW]) { vload<V, VW>(x + e, o); }, q);
        vstore<V, VW>(y + c, q);
    });
}

template <typename V, int VW>
__global__ __launch_bounds__(kKB) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_resid_t(Dims d, int nblk, const V *__restrict__ a, const V *__restrict__ b,
                                                 const V *__restrict__ y, V *__restrict__ r, double *partials,
                                                 unsigned *counter, DevScalars *sc, int restart)
{
    k_resid_body<VW>(d, nblk, a, b, y, r, partials, counter, sc, restart);
}

void launch_spmv(const Dims &d, int nblk, const double *a, const double *x, double *y, hipStream_t st)
{
    RT_DISPATCH_VW(double, pick_vw<double>(d), k_spmv_t, dim3(nblk), dim3(kKB), 0, st, d, nblk, a, x, y);
}

void launch_spmv32(const Dims &d, int nblk, const float *a, const float *x, float *y, hipStream_t st)
{
    RT_DISPATCH_VW(float, pick_vw<float>(d), k_spmv_t, dim3(nblk), dim3(kKB), 0, st, d, nblk, a, x, y);
}

void launch_norm2(const Dims &d, int nblk, const double *x, double *partials, unsigned *counter,
                  DevScalars *sc, hipStream_t st)
{
    hipLaunchKernelGGL(k_norm2, dim3(nblk), dim3(kKB), 0, st, d, nblk, x, partials, counter, sc);
}

void launch_resid(const Dims &d, int nblk, const double *a, const double *b, const double *y,
                  double *r, double *partials, unsigned *counter, DevScalars *sc, int restart, hipStream_t st)
{
    RT_DISPATCH_VW(double, pick_vw<double>(d), k_resid_t, dim3(nblk), dim3(kKB), 0, st, d, nblk, a, b, y, r,
                   partials, counter, sc, restart);
}

// The direction pass alternates its sweep direction between iterations and the update
// sweeps against it with non-temporal streams: each direction pass then starts on the
// rows whose coefficients and vectors the previous one touched last, which the update
// has not pushed out of the Infinity Cache, and the update starts on the direction
// pass's last p and q.
template <typename V>
static void cg_iter(const Dims &d, int nblk, int nblk_upd, const V *a, V *y, V *r, V *pold, V *pnew, V *q,
                    double *partials, unsigned *counter, DevScalars *sc, hipStream_t st, const hipEvent_t *ev, int odd)
{
    const int vw = pick_vw<V>(d);
    Dims dd = d, du = d;
    dd.rev = odd;
    du.rev = !odd;
    if (ev) (void)hipEventRecord(ev[0], st);
    RT_DISPATCH_VW(V, vw, k_cg_dir, dim3(nblk), dim3(kKB), 0, st, dd, nblk, a, r, pold, pnew, q, partials, counter,
                   sc);
    if (ev) (void)hipEventRecord(ev[1], st);
    RT_DISPATCH_VW(V, vw, k_cg_upd_nt, dim3(nblk_upd), dim3(kKB), 0, st, du, nblk_upd, y, pnew, r, q, partials,
                   counter, sc);
    if (ev) (void)hipEventRecord(ev[2], st);
}

void launch_cg_iter64(const Dims &d, int nblk, int nblk_upd, const double *a, double *y, double *r, double *pold,
                      double *pnew, double *q, double *partials, unsigned *counter, DevScalars *sc,
                      hipStream_t st, const hipEvent_t *ev, int odd)
{
    cg_iter<double>(d, nblk, nblk_upd, a, y, r, pold, pnew, q, partials, counter, sc, st, ev, odd);
}

void launch_cg_iter32(const Dims &d, int nblk, int nblk_upd, const float *a, float *x, float *r, float *pold,
                      float *pnew, float *q, double *partials, unsigned *counter, DevScalars *sc,
                      hipStream_t st, const hipEvent_t *ev, int odd)
{
    cg_iter<float>(d, nblk, nblk_upd, a, x, r, pold, pnew, q, partials, counter, sc, st, ev, odd);
}

void launch_reliable(const Dims &d, int nblk, const double *r, float *r32, float *x32, double *partials,
                     unsigned *counter, DevScalars *sc, int restart, hipStream_t st)
{
    hipLaunchKernelGGL(k_reliable, dim3(nblk), dim3(kKB), 0, st, d, nblk, r, r32, x32, partials, counter,
                       sc, restart);
}

void launch_fcg_dir(const Dims &d, int nblk, const float *a, const float *z, const float *pold, const float *r,
                    float *pnew, float *q, double *partials, unsigned *counter, DevScalars *sc, hipStream_t st)
{
    if (d.nr % 4 == 0)
        hipLaunchKernelGGL(k_fcg_dir<4>, dim3(nblk), dim3(kKB), 0, st, d, nblk, a, z, pold, r, pnew, q, partials,
                           counter, sc);
    else
        hipLaunchKernelGGL(k_fcg_dir<1>, dim3(nblk), dim3(kKB), 0, st, d, nblk, a, z, pold, r, pnew, q, partials,
                           counter, sc);
}

void launch_fcg_beta(const Dims &d, int nblk, const float *z, const float *q, double *partials, unsigned *counter,
                     DevScalars *sc, hipStream_t st)
{
    hipLaunchKernelGGL(k_fcg_beta, dim3(nblk), dim3(kKB), 0, st, d, nblk, z, q, partials, counter, sc);
}

void launch_cg_upd32(const Dims &d, int nblk, float *x, const float *p, float *r, const float *q, double *partials,
                     unsigned *counter, DevScalars *sc, hipStream_t st)
{
    const int vw = pick_vw<float>(d);
    RT_DISPATCH_VW(float, vw, k_cg_upd, dim3(nblk), dim3(kKB), 0, st, d, nblk, x, p, r, q, partials, counter, sc);
}

void launch_norm2_rr32(const Dims &d, int nblk, const float *x, double *partials, unsigned *counter,
                       DevScalars *sc, hipStream_t st)
{
    hipLaunchKernelGGL(k_norm2_rr32, dim3(nblk), dim3(kKB), 0, st, d, nblk, x, partials, counter, sc);
}

void launch_rms_scale(long n, const DevScalars *sc, double *scale, hipStream_t st)
{
    hipLaunchKernelGGL(k_rms_scale, dim3(1), dim3(64), 0, st, n, sc, scale);
}

void launch_fold(long n, const float *x32, double *y, hipStream_t st)
{
    hipLaunchKernelGGL(k_fold, dim3((unsigned)((n + kKB - 1) / kKB)), dim3(kKB), 0, st, n, x32, y);
}


// ------------------------------------------------------ red-black reduced system
//
// Colour the cells black ((i + j + k) even) and red (odd).  The 7-point operator only
// couples cells of different colours (with N_phi even or 1, so that the periodic phi
// seam also joins opposite colours), so in that ordering A^ = [I B; B^T I] with B the
// red-black couplings.  Eliminating the red unknowns leaves
//   S y_b = b_b - B^T b_r,   S = I - B^T B,   then   y_r = b_r - B y_b,
// with S symmetric positive definite and cond(S) = cond(A^) / (1 + ||B||)^2, about a
// quarter: CG on S needs about half the iterations of CG on A^, and one product with S
// (a pass over the red cells, t = B p, then one over the black cells, q = p - B^T t)
// moves about the bytes of one product with A^, because each pass reads every face
// coefficient once and half of the vector entries (the red pass forms p and stores it
// for the black pass and the update).  The residual of S is the residual
// of A^ once y_r is formed, so the stopping test is unchanged.
// Layout: each colour is stored compactly with H = N_r / 2 cells per radial row; the
// half index g = h + H (j + N_theta k) holds the cell i = 2h + par of row (j, k), par =
// (j + k) & 1 for black and 1 - that for red.  ab[col][dir][g] is the outward r /
// theta / phi coefficient of that cell (col 0 black, 1 red).  The kernels run over the
// half grid Dims{H, N_theta, N_phi} with the row mapping of for_segments.

// acc = sum over the six neighbours (all of the other colour) of coefficient x value,
// for the VW cells h0 .. h0+VW-1 of row rw whose full radial index is 2h + par.  own /
// oth are the outward coefficients ([3][n_half]) of this colour and of the other one;
// seg(e, o) loads VW values of the other colour's vector at half index e, one(e) one
// value.  Summation order: +r, -r, +theta, -theta, +phi, -phi.
template <typename V, int VW, typename Seg, typename One>
__device__ __forceinline__ void rb_couple(const Dims &dh, const Row &rw, int h0, int par, const V *__restrict__ own,
                                          const V *__restrict__ oth, Seg &&seg, One &&one, V (&acc)[VW])
{
    const long nh = dh.n;
    const int H = dh.nr;
    const long g = rw.base + h0;
    // radial: the right neighbour of cell m (i + 1) is the other colour's half h0+m+par,
    // the left one (i - 1) is h0+m-1+par; the element beyond the aligned segment is
    // h0+VW (par = 1, clamped at the row end where the own coefficient is 0) or h0-1
    // (par = 0, absent at the row start, where the coefficient is masked)
    V x[VW], co[VW], cl[VW];
    seg(g, x);
    vload<V, VW>(own + g, co);
    vload<V, VW>(oth + g, cl);
    const bool hasl = h0 > 0;
    const long ge = par ? (h0 + VW < H ? g + VW : g + VW - 1) : (hasl ? g - 1 : g);
    const V xe = one(ge);
    const V ce = (!par && hasl) ? oth[ge] : V(0);
    V xjp[VW], xjm[VW], xkp[VW], xkm[VW], ctp[VW], ctm[VW], cpp[VW], cpm[VW];
    const long gjm = rw.jm ? g - H : g;
    seg(rw.jp ? g + H : g, xjp);  // the own theta coefficient is 0 in the last polar row
    seg(gjm, xjm);
    seg(g + rw.kp, xkp);          // the offsets are 0 when N_phi = 1 (coefficients 0 then)
    seg(g + rw.km, xkm);
    vload<V, VW>(own + nh + g, ctp);
    vload<V, VW>(oth + nh + gjm, ctm);
    vload<V, VW>(own + 2 * nh + g, cpp);
    vload<V, VW>(oth + 2 * nh + g + rw.km, cpm);
    const V mjm = (V)rw.jm;
#pragma unroll
    for (int m = 0; m < VW; m++) {
        const V right = par ? (m + 1 < VW ? x[m + 1] : xe) : x[m];
        const V left = par ? x[m] : (m > 0 ? x[m - 1] : xe);
        const V cleft = par ? cl[m] : (m > 0 ? cl[m - 1] : ce);
        V v = co[m] * right;
        v += cleft * left;
        v += ctp[m] * xjp[m];
        v += (ctm[m] * mjm) * xjm[m];
        v += cpp[m] * xkp[m];
        v += cpm[m] * xkm[m];
        acc[m] = v;
    }
}

// Red pass of a CG iteration on S: t_r = B p with p_b = r_b + beta p_old_b formed at
// the neighbours.  The black segment at the same half indices as the red one (its
// aligned radial neighbours) is stored as p_b: the segments of the pass cover every
// black half index once, so the black pass reads p_b instead of forming it again.
template <typename V, int VW>
__global__ __launch_bounds__(kKB) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_rb_red_dir(
    Dims dh, int nblk, const V *__restrict__ ab, const V *__restrict__ r, const V *__restrict__ pold,
    V *__restrict__ pnew, V *__restrict__ t, DevScalars *sc)
{
    if (sc->done) return;
    const V beta = (V)sc->beta;
    const V *own = ab + 3 * dh.n, *oth = ab;
    for_segments<VW>(dh, nblk, [&](const Row &rw, int h0) {
        const long g = rw.base + h0;
        V ps[VW], acc[VW];
        dir_seg<V, VW>(r, pold, beta, g, ps);
        vstore<V, VW>(pnew + g, ps);
        rb_couple<V, VW>(dh, rw, h0, 1 - rw.par, own, oth,
                         [&](long e, V(&o)[VW]) { dir_seg<V, VW>(r, pold, beta, e, o); },
                         [&](long e) { return dir_one(r, pold, beta, e); }, acc);
        vstore<V, VW>(t + g, acc);
    });
}

// Black pass: q_b = p_b - B^T t_r (p_b from the red pass), pq = p.q, alpha = rr / pq.
template <typename V, int VW>
__global__ __launch_bounds__(kKB) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_rb_black_dir(
    Dims dh, int nblk, const V *__restrict__ ab, const V *__restrict__ p, const V *__restrict__ t,
    V *__restrict__ q, double *partials, unsigned *counter, DevScalars *sc)
{
    if (sc->done) return;
    __shared__ double sh[kKB / 64];
    const V *own = ab, *oth = ab + 3 * dh.n;
    const long L = logical_block(nblk);
    double acc = 0.0;
    for_segments<VW>(dh, nblk, [&](const Row &rw, int h0) {
        const long g = rw.base + h0;
        V pv[VW], bt[VW], qv[VW];
        vload<V, VW>(p + g, pv);
        rb_couple<V, VW>(dh, rw, h0, rw.par, own, oth, [&](long e, V(&o)[VW]) { vload<V, VW>(t + e, o); },
                         [&](long e) { return t[e]; }, bt);
#pragma unroll
        for (int m = 0; m < VW; m++) qv[m] = pv[m] - bt[m];
        vstore<V, VW>(q + g, qv);
#pragma unroll
        for (int m = 0; m < VW; m++) acc += (double)pv[m] * (double)qv[m];
    });
    double bs = block_sum(acc, sh), tot;
    if (finish_reduce(bs, L, nblk, partials, counter, sh, &tot) && threadIdx.x == 0) {
        sc->pq = tot;
        sc->alpha = sc->rr / tot;
    }
}

// Float64 red pass: out_r = u_r + sgn (B x_b) (u may be NULL): t = B y_b for a true
// residual, y_r = b_r - B y_b for the back substitution.
template <typename V, int VW>
__global__ __launch_bounds__(kKB) void k_rb_red_apply(Dims dh, int nblk, const double *__restrict__ ab,
                                                      const double *__restrict__ x, const double *__restrict__ u,
                                                      double sgn, double *__restrict__ out)
{
    const double *own = ab + 3 * dh.n, *oth = ab;
    for_segments<VW>(dh, nblk, [&](const Row &rw, int h0) {
        const long g = rw.base + h0;
        double acc[VW], uv[VW];
        rb_couple<double, VW>(dh, rw, h0, 1 - rw.par, own, oth,
                              [&](long e, double(&o)[VW]) { vload<double, VW>(x + e, o); },
                              [&](long e) { return x[e]; }, acc);
        if (u) vload<double, VW>(u + g, uv);
#pragma unroll
        for (int m = 0; m < VW; m++) acc[m] = (u ? uv[m] : 0.0) + sgn * acc[m];
        vstore<double, VW>(out + g, acc);
    });
}

// Float64 black pass: out_b = u_b - x_b + sgn (B^T t_r) (x may be NULL) and res2 =
// out.out, with the restart semantics of k_resid.  r_b = bb - y_b + B^T (B y_b) is the
// residual of S; bb = b_b - B^T b_r the reduced right-hand side.
template <typename V, int VW>
__global__ __launch_bounds__(kKB) void k_rb_black_apply(Dims dh, int nblk, const double *__restrict__ ab,
                                                        const double *__restrict__ t, const double *__restrict__ u,
                                                        const double *__restrict__ x, double sgn,
                                                        double *__restrict__ out, double *partials, unsigned *counter,
                                                        DevScalars *sc, int restart)
{
    __shared__ double sh[kKB / 64];
    const double *own = ab, *oth = ab + 3 * dh.n;
    const long L = logical_block(nblk);
    double acc = 0.0;
    for_segments<VW>(dh, nblk, [&](const Row &rw, int h0) {
        const long g = rw.base + h0;
        double bt[VW], uv[VW], xv[VW];
        rb_couple<double, VW>(dh, rw, h0, rw.par, own, oth,
                              [&](long e, double(&o)[VW]) { vload<double, VW>(t + e, o); },
                              [&](long e) { return t[e]; }, bt);
        vload<double, VW>(u + g, uv);
        if (x) vload<double, VW>(x + g, xv);
#pragma unroll
        for (int m = 0; m < VW; m++) {
            double v = uv[m] - (x ? xv[m] : 0.0);
            v += sgn * bt[m];
            uv[m] = v;
            acc += v * v;
        }
        vstore<double, VW>(out + g, uv);
    });
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

// Colour split of the assembled operator: ab[col][dir][g] (and its float copy) from the
// natural outward coefficients a[dir][c]; one thread per natural cell.
__global__ __launch_bounds__(kKB) void k_rb_split(Dims d, const double *__restrict__ a, double *__restrict__ ab,
                                                  float *__restrict__ ab32)
{
    const long c = (long)blockIdx.x * kKB + threadIdx.x;
    if (c >= d.n) return;
    const int i = (int)(c % d.nr);
    const long row = c / d.nr;
    const int j = (int)(row % d.nt), k = (int)(row / d.nt);
    const int col = (i + j + k) & 1;
    const long nh = d.n / 2, g = (i >> 1) + (long)(d.nr / 2) * row;
#pragma unroll
    for (int dir = 0; dir < 3; dir++) {
        const double v = a[dir * d.n + c];
        ab[(col * 3 + dir) * nh + g] = v;
        ab32[(col * 3 + dir) * nh + g] = (float)v;
    }
}

// Natural vector x <-> its black and red halves (xb / xr may be NULL when gathering).
__global__ __launch_bounds__(kKB) void k_rb_gather(Dims d, const double *__restrict__ x, double *__restrict__ xb,
                                                   double *__restrict__ xr)
{
    const long c = (long)blockIdx.x * kKB + threadIdx.x;
    if (c >= d.n) return;
    const int i = (int)(c % d.nr);
    const long row = c / d.nr;
    const int j = (int)(row % d.nt), k = (int)(row / d.nt);
    const long g = (i >> 1) + (long)(d.nr / 2) * row;
    double *dst = ((i + j + k) & 1) ? xr : xb;
    if (dst) dst[g] = x[c];
}

__global__ __launch_bounds__(kKB) void k_rb_scatter(Dims d, const double *__restrict__ xb,
                                                    const double *__restrict__ xr, double *__restrict__ x)
{
    const long c = (long)blockIdx.x * kKB + threadIdx.x;
    if (c >= d.n) return;
    const int i = (int)(c % d.nr);
    const long row = c / d.nr;
    const int j = (int)(row % d.nt), k = (int)(row / d.nt);
    const long g = (i >> 1) + (long)(d.nr / 2) * row;
    x[c] = ((i + j + k) & 1) ? xr[g] : xb[g];
}

Dims rb_half(const Dims &d)
{
    return Dims{d.nr / 2, d.nt, d.np, d.n / 2, (long)(d.nr / 2) * d.nt};
}

static unsigned grid1(long n) { return (unsigned)((n + kKB - 1) / kKB); }

void launch_rb_split(const Dims &d, const double *a, double *ab, float *ab32, hipStream_t st)
{
    hipLaunchKernelGGL(k_rb_split, dim3(grid1(d.n)), dim3(kKB), 0, st, d, a, ab, ab32);
}

void launch_rb_gather(const Dims &d, const double *x, double *xb, double *xr, hipStream_t st)
{
    hipLaunchKernelGGL(k_rb_gather, dim3(grid1(d.n)), dim3(kKB), 0, st, d, x, xb, xr);
}

void launch_rb_scatter(const Dims &d, const double *xb, const double *xr, double *x, hipStream_t st)
{
    hipLaunchKernelGGL(k_rb_scatter, dim3(grid1(d.n)), dim3(kKB), 0, st, d, xb, xr, x);
}

void launch_rb_red_apply(const Dims &dh, int nblk, const double *ab, const double *x, const double *u, double sgn,
                         double *out, hipStream_t st)
{
    RT_DISPATCH_VW(double, pick_vw<double>(dh), k_rb_red_apply, dim3(nblk), dim3(kKB), 0, st, dh, nblk, ab, x, u,
                   sgn, out);
}

void launch_rb_black_apply(const Dims &dh, int nblk, const double *ab, const double *t, const double *u,
                           const double *x, double sgn, double *out, double *partials, unsigned *counter,
                           DevScalars *sc, int restart, hipStream_t st)
{
    RT_DISPATCH_VW(double, pick_vw<double>(dh), k_rb_black_apply, dim3(nblk), dim3(kKB), 0, st, dh, nblk, ab, t,
                   u, x, sgn, out, partials, counter, sc, restart);
}

// Sweep directions and the Infinity Cache (256 MB, which holds the last ~20 % of what a
// pass at 512x256x512 touched): the red pass sweeps forward, the black pass backward, so
// it starts on the rows whose p, t and six coefficient arrays the red pass touched last;
// the update sweeps forward, starting on the black pass's last p and q, with
// non-temporal streams, so it leaves the black pass's last rows -- the same coefficient
// arrays and p -- in the cache for the next red pass, which starts there.  At
// 512x256x512 (float, rocprofv3 medians): red 263 -> 245 us, black 239 -> 227 us,
// update 144 -> 138 us against one direction for all three passes and plain streams;
// the L2-miss traffic is the same.  (Non-temporal loads of t in the black pass are
// slower: t is read again by the neighbouring rows, from L2.)
template <typename V>
static void rb_iter(const Dims &dh, int nblk, int nblk_upd, const V *ab, V *y, V *r, V *pold, V *pnew, V *q, V *t,
                    double *partials, unsigned *counter, DevScalars *sc, hipStream_t st, const hipEvent_t *ev)
{
    const int vw = pick_vw<V>(dh);
    Dims da = dh, db = dh;
    da.rev = 0;
    db.rev = 1;
    if (ev) (void)hipEventRecord(ev[0], st);
    RT_DISPATCH_VW(V, vw, k_rb_red_dir, dim3(nblk), dim3(kKB), 0, st, da, nblk, ab, r, pold, pnew, t, sc);
    if (ev) (void)hipEventRecord(ev[3], st);
    RT_DISPATCH_VW(V, vw, k_rb_black_dir, dim3(nblk), dim3(kKB), 0, st, db, nblk, ab, (const V *)pnew, (const V *)t, q,
                   partials, counter, sc);
    if (ev) (void)hipEventRecord(ev[1], st);
    RT_DISPATCH_VW(V, vw, k_cg_upd_nt, dim3(nblk_upd), dim3(kKB), 0, st, da, nblk_upd, y, pnew, r, q, partials,
                   counter, sc);
    if (ev) (void)hipEventRecord(ev[2], st);
}

void launch_rb_iter64(const Dims &dh, int nblk, int nblk_upd, const double *ab, double *y, double *r, double *pold,
                      double *pnew, double *q, double *t, double *partials, unsigned *counter, DevScalars *sc,
                      hipStream_t st, const hipEvent_t *ev)
{
    rb_iter<double>(dh, nblk, nblk_upd, ab, y, r, pold, pnew, q, t, partials, counter, sc, st, ev);
}

void launch_rb_iter32(const Dims &dh, int nblk, int nblk_upd, const float *ab, float *x, float *r, float *pold,
                      float *pnew, float *q, float *t, double *partials, unsigned *counter, DevScalars *sc,
                      hipStream_t st, const hipEvent_t *ev)
{
    rb_iter<float>(dh, nblk, nblk_upd, ab, x, r, pold, pnew, q, t, partials, counter, sc, st, ev);
}

// ------------------------------------------- one-workgroup reduced CG (small grids)
//
// On grids of a few thousand cells each kernel of an iteration lasts a few
// microseconds and the launches, not the bytes, set the time (the paper's own runs are
// 2-D grids of this size).  Here one workgroup of kSB threads runs the float64 CG
// iterations on S by itself: the direction p (black) and the product t = B p (red) --
// the two vectors whose neighbours are read -- live in LDS; the thread's own entries of
// r, y, q, p and t and each of its cells' couplings (six coefficients and neighbour
// indices per colour, read once per launch) live in registers; and each iteration's two
// dot products are workgroup sums in a fixed order.  Thread tid owns the half indices tid + c kSB,
// c < CPT <= 2 (at most 2048 black cells: beyond that the couplings no longer fit the
// registers, and from L2 a single CU streams them no faster than the multi-block
// kernels run).  Every entry is summed as in rb_couple (same terms, same order); only
// the summation order of the dot products differs from the multi-block kernels.  At
// most m iterations per launch; the state (y, r, p and the scalars) is read at the
// start and written back at the end, so launches chain like the multi-block chunks.
constexpr int kSB = 1024;

// A lane permutation inside each row of 16 lanes (DPP), applied to a double.
template <int Ctrl>
__device__ __forceinline__ double dpp_d(double v)
{
    int2 t = *reinterpret_cast<int2 *>(&v);
    t.x = __builtin_amdgcn_update_dpp(0, t.x, Ctrl, 0xF, 0xF, false);
    t.y = __builtin_amdgcn_update_dpp(0, t.y, Ctrl, 0xF, 0xF, false);
    return *reinterpret_cast<double *>(&t);
}

// Sum over the workgroup; the same value in every thread.  Inside a wave: four DPP
// butterfly steps inside each row of 16 lanes (swap neighbours, swap pairs, mirror
// halves of 8, mirror the row; each step adds a lane and its partner, a + b = b + a,
// so every lane of a row ends with the same row total), then the four row totals read
// into scalars and added in a fixed order.  Across the workgroup every thread adds the
// wave totals in index order, so the convergence test is uniform.  (A pairwise tree
// over the 16 totals was slower: its 16 live doubles pushed the kernel's registers.)
__device__ __forceinline__ double wg_sum(double v, double *sh)
{
    v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_d<0x141>(v);  // row_half_mirror
    v += dpp_d<0x140>(v);  // row_mirror
    const double w = (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = w;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kSB / 64; i++) t += sh[i];
    return t;
}

// The couplings of one cell to its six neighbours of the other colour, in the terms and
// order of rb_couple with VW = 1: right, left, +theta, -theta, +phi, -phi (an absent
// neighbour has index g and coefficient 0).  One of the two radial neighbours is the
// other colour's cell at the same half index g, whose value the thread holds in a
// register (it owns both cells at g); e[0] is the other one's index and `right` tells
// which side it is on.
struct Cpl {
    double w[6];
    int e[6];
    bool right;
};

__device__ __forceinline__ Cpl couplings(const Dims &dh, const Row &rw, int h0, int par, const double *__restrict__ own,
                                         const double *__restrict__ oth)
{
    const long nh = dh.n;
    const int H = dh.nr;
    const long g = rw.base + h0;
    const bool hasl = h0 > 0;
    const long ge = par ? (h0 + 1 < H ? g + 1 : g) : (hasl ? g - 1 : g);
    const long gjm = rw.jm ? g - H : g;
    Cpl c;
    c.w[0] = own[g];
    c.w[1] = par ? oth[g] : (hasl ? oth[ge] : 0.0);
    c.e[0] = (int)ge;  // the radial neighbour that is not at g (at the row ends ge = g)
    c.right = par != 0;
    c.e[1] = (int)g;   // unused
    c.w[2] = own[nh + g];
    c.e[2] = (int)(rw.jp ? g + H : g);
    c.w[3] = oth[nh + gjm] * (double)rw.jm;
    c.e[3] = (int)gjm;
    c.w[4] = own[2 * nh + g];
    c.e[4] = (int)(g + rw.kp);
    c.w[5] = oth[2 * nh + g + rw.km];
    c.e[5] = (int)(g + rw.km);
    return c;
}

// xg: the value at index g (from the register that holds it)
__device__ __forceinline__ double couple(const Cpl &c, const double *x, double xg)
{
    const double xo = x[c.e[0]];
    double v = c.w[0] * (c.right ? xo : xg);
    v += c.w[1] * (c.right ? xg : xo);
    v += c.w[2] * x[c.e[2]];
    v += c.w[3] * x[c.e[3]];
    v += c.w[4] * x[c.e[4]];
    v += c.w[5] * x[c.e[5]];
    return v;
}

template <int CPT>
__global__ __launch_bounds__(kSB) void k_rb_cg_block(Dims dh, const double *__restrict__ ab, double *__restrict__ y,
                                                    double *__restrict__ r, double *__restrict__ p, int m,
                                                    DevScalars *sc)
{
    extern __shared__ double lds[];
    // two buffers for the two sums of an iteration: a thread can only overwrite one
    // after every thread has passed the barrier of the other, i.e. has read it
    __shared__ double sha[kSB / 64], shb[kSB / 64];
    if (sc->done) return;
    const long nh = dh.n;
    const int H = dh.nr;
    double *ps = lds, *ts = lds + nh;
    const double *blk = ab, *red = ab + 3 * nh;
    Cpl cr[CPT], cb[CPT];  // couplings of the red and of the black cell at half index g
    int gi[CPT];
    bool own[CPT];
    double rv[CPT], yv[CPT], pr[CPT], tr[CPT];  // r, y, p (black) and t (red) at g
#pragma unroll
    for (int c = 0; c < CPT; c++) {
        const long g = threadIdx.x + (long)c * kSB;
        own[c] = g < nh;
        gi[c] = (int)g;
        rv[c] = yv[c] = pr[c] = tr[c] = 0.0;
        if (!own[c]) {
            cr[c] = cb[c] = Cpl{};
            continue;
        }
        const long row = g / H;
        const int j = (int)(row % dh.nt), k = (int)(row / dh.nt);
        Row rw;
        rw.base = row * H;
        rw.jp = j + 1 < dh.nt;
        rw.jm = j > 0;
        rw.kk = dh.np > 1;
        rw.kp = (k + 1 < dh.np) ? dh.plane : -(long)(dh.np - 1) * dh.plane;
        rw.km = (k > 0) ? -dh.plane : (long)(dh.np - 1) * dh.plane;
        rw.par = (j + k) & 1;
        const int h0 = (int)(g - rw.base);
        cr[c] = couplings(dh, rw, h0, 1 - rw.par, red, blk);
        cb[c] = couplings(dh, rw, h0, rw.par, blk, red);
        rv[c] = r[g];
        yv[c] = y[g];
        pr[c] = p[g];
    }
    double rr = sc->rr, beta = sc->beta, pq = sc->pq, alpha = sc->alpha;
    const double th = sc->thresh2;
    int it = 0, done = 0;
    while (it < m && !done) {
        // p = r + beta p (each thread its own entries, kept in registers too)
#pragma unroll
        for (int c = 0; c < CPT; c++)
            if (own[c]) {
                pr[c] = fma(beta, pr[c], rv[c]);
                ps[gi[c]] = pr[c];
            }
        __syncthreads();
        // red: t = B p
#pragma unroll
        for (int c = 0; c < CPT; c++)
            if (own[c]) {
                tr[c] = couple(cr[c], ps, pr[c]);
                ts[gi[c]] = tr[c];
            }
        __syncthreads();
        // black: q = p - B^T t, p.q
        double qv[CPT], part = 0.0;
#pragma unroll
        for (int c = 0; c < CPT; c++) {
            qv[c] = 0.0;
            if (own[c]) {
                qv[c] = pr[c] - couple(cb[c], ts, tr[c]);
                part += pr[c] * qv[c];
            }
        }
        pq = wg_sum(part, sha);
        alpha = rr / pq;
        part = 0.0;
#pragma unroll
        for (int c = 0; c < CPT; c++)
            if (own[c]) {
                yv[c] = fma(alpha, pr[c], yv[c]);
                rv[c] = fma(-alpha, qv[c], rv[c]);
                part += rv[c] * rv[c];
            }
        const double rn = wg_sum(part, shb);
        beta = rn / rr;
        rr = rn;
        it++;
        if (rn <= th || !(rn == rn)) done = 1;
    }
#pragma unroll
    for (int c = 0; c < CPT; c++)
        if (own[c]) {
            r[gi[c]] = rv[c];
            y[gi[c]] = yv[c];
            p[gi[c]] = pr[c];
        }
    if (threadIdx.x == 0) {
        sc->rr = rr;
        sc->beta = beta;
        sc->pq = pq;
        sc->alpha = alpha;
        sc->iters += it;
        sc->done = done;
    }
}

__global__ void k_solve_init(DevScalars *sc, double tol2)
{
    if (threadIdx.x != 0) return;
    const double bb = sc->res2 == 0.0 ? 1.0 : sc->res2;
    sc->bnorm2 = bb;
    sc->thresh2 = tol2 * bb;
    sc->done = 0;
    sc->iters = 0;
    sc->beta = 0.0;
}

void launch_solve_init(DevScalars *sc, double tol2, hipStream_t st)
{
    hipLaunchKernelGGL(k_solve_init, dim3(1), dim3(64), 0, st, sc, tol2);
}

int rb_block_cpt(const Dims &dh)
{
    const long c = (dh.n + kSB - 1) / kSB;
    return c <= 1 ? 1 : c <= 2 ? 2 : 0;
}

bool launch_rb_cg_block(const Dims &dh, const double *ab, double *y, double *r, double *p, int m, DevScalars *sc,
                        hipStream_t st)
{
    const int cpt = rb_block_cpt(dh);
    const size_t lds = 2 * (size_t)dh.n * sizeof(double);  // at most 32 KiB
    if (cpt == 0 || m <= 0) return false;
    if (cpt == 1)
        hipLaunchKernelGGL(k_rb_cg_block<1>, dim3(1), dim3(kSB), lds, st, dh, ab, y, r, p, m, sc);
    else
        hipLaunchKernelGGL(k_rb_cg_block<2>, dim3(1), dim3(kSB), lds, st, dh, ab, y, r, p, m, sc);
    return true;
}

// --------------------------------------- radial-line block-Jacobi comparator
//
// The block-Jacobi class of preconditioner the paper uses (with ILU inside the blocks),
// in the form that suits a GPU: the blocks are the radial rows, whose tridiagonal
// couplings tridiag(a_r[i-1], 1, a_r[i]) are factorised exactly (Thomas: c_i and 1/m_i
// once per system) and solved per application.  One thread per row walks it outward
// and back; the rows of a wavefront are N_r apart in memory, so each lane streams its
// own row through the caches (a comparator, not tuned).

// c[i] = a_r[i] / m_i, im[i] = 1 / m_i with m_0 = 1, m_i = 1 - a_r[i-1] c[i-1].
__global__ __launch_bounds__(kKB) void k_line_factor(Dims d, const double *__restrict__ a, double *__restrict__ c,
                                                     double *__restrict__ im)
{
    const long rows = (long)d.nt * d.np;
    for (long row = (long)blockIdx.x * kKB + threadIdx.x; row < rows; row += (long)gridDim.x * kKB) {
        const long b = row * d.nr;
        double cp = 0.0, ap = 0.0;
        for (int i = 0; i < d.nr; i++) {
            const double m = 1.0 - ap * cp;
            const double ai = a[b + i];
            cp = ai / m;
            c[b + i] = cp;
            im[b + i] = 1.0 / m;
            ap = ai;
        }
    }
}

// z = M^-1 r (tridiagonal solve per radial row), rz = r.z; beta = rz / rz_prev (0 after
// a restart), rr = rz for the direction kernel.
__global__ __launch_bounds__(kKB) void k_line_solve(Dims d, int nblk, const double *__restrict__ a,
                                                    const double *__restrict__ c, const double *__restrict__ im,
                                                    const double *__restrict__ r, double *__restrict__ z,
                                                    double *partials, unsigned *counter, DevScalars *sc, int restart)
{
    if (sc->done) return;
    __shared__ double sh[kKB / 64];
    const long rows = (long)d.nt * d.np;
    double acc = 0.0;
    for (long row = (long)blockIdx.x * kKB + threadIdx.x; row < rows; row += (long)nblk * kKB) {
        const long b = row * d.nr;
        double dp = 0.0, ap = 0.0;
        for (int i = 0; i < d.nr; i++) {  // forward: d_i = (r_i - a_(i-1) d_(i-1)) / m_i
            dp = (r[b + i] - ap * dp) * im[b + i];
            z[b + i] = dp;
            ap = a[b + i];
        }
        double zn = 0.0;
        for (int i = d.nr - 1; i >= 0; i--) {  // backward: z_i = d_i - c_i z_(i+1)
            zn = z[b + i] - c[b + i] * zn;
            z[b + i] = zn;
            acc += r[b + i] * zn;
        }
    }
    const long L = logical_block(nblk);
    double bs = block_sum(acc, sh), tot;
    if (finish_reduce(bs, L, nblk, partials, counter, sh, &tot) && threadIdx.x == 0) {
        sc->beta = (restart || !(sc->rr > 0.0)) ? 0.0 : tot / sc->rr;
        sc->rr = tot;
    }
}

// Preconditioned update: y += alpha p, r -= alpha q, res2 = r.r, done when res2 <= thresh2.
template <int VW>
__global__ __launch_bounds__(kKB) void k_pcg_upd(Dims d, int nblk, double *__restrict__ y,
                                                 const double *__restrict__ p, double *__restrict__ r,
                                                 const double *__restrict__ q, double *partials, unsigned *counter,
                                                 DevScalars *sc)
{
    if (sc->done) return;
    __shared__ double sh[kKB / 64];
    const double alpha = sc->alpha;
    const long L = logical_block(nblk);
    double acc = 0.0;
    for_segments<VW>(d, nblk, [&](const Row &rw, int i) {
        const long c = rw.base + i;
        double yv[VW], pv[VW], rv[VW], qv[VW];
        vload<double, VW>(y + c, yv);
        vload<double, VW>(p + c, pv);
        vload<double, VW>(r + c, rv);
        vload<double, VW>(q + c, qv);
#pragma unroll
        for (int m = 0; m < VW; m++) {
            yv[m] = fma(alpha, pv[m], yv[m]);
            rv[m] = fma(-alpha, qv[m], rv[m]);
            acc += rv[m] * rv[m];
        }
        vstore<double, VW>(y + c, yv);
        vstore<double, VW>(r + c, rv);
    });
    double bs = block_sum(acc, sh), tot;
    if (finish_reduce(bs, L, nblk, partials, counter, sh, &tot) && threadIdx.x == 0) {
        sc->res2 = tot;
        sc->iters += 1;
        if (tot <= sc->thresh2 || !(tot == tot)) sc->done = 1;
    }
}

void launch_line_factor(const Dims &d, int nblk, const double *a, double *c, double *im, hipStream_t st)
{
    hipLaunchKernelGGL(k_line_factor, dim3(nblk), dim3(kKB), 0, st, d, a, c, im);
}

void launch_line_solve(const Dims &d, int nblk, const double *a, const double *c, const double *im, const double *r,
                       double *z, double *partials, unsigned *counter, DevScalars *sc, int restart, hipStream_t st)
{
    hipLaunchKernelGGL(k_line_solve, dim3(nblk), dim3(kKB), 0, st, d, nblk, a, c, im, r, z, partials, counter, sc,
                       restart);
}

// The rest of a preconditioned CG iteration once z = M^-1 r and beta are known:
// p = z + beta p_old, q = A^ p, alpha; y, r update and r.r.
void launch_pcg_dir_upd(const Dims &d, int nblk, int nblk_upd, const double *a, const double *z, double *y, double *r,
                        double *pold, double *pnew, double *q, double *partials, unsigned *counter, DevScalars *sc,
                        hipStream_t st, const hipEvent_t *ev)
{
    const int vw = pick_vw<double>(d);
    RT_DISPATCH_VW(double, vw, k_cg_dir, dim3(nblk), dim3(kKB), 0, st, d, nblk, a, z, pold, pnew, q, partials,
                   counter, sc);
    if (ev) (void)hipEventRecord(ev[1], st);
    switch (vw) {
    case 8: hipLaunchKernelGGL(k_pcg_upd<8>, dim3(nblk_upd), dim3(kKB), 0, st, d, nblk_upd, y, pnew, r, q, partials,
                               counter, sc); break;
    case 4: hipLaunchKernelGGL(k_pcg_upd<4>, dim3(nblk_upd), dim3(kKB), 0, st, d, nblk_upd, y, pnew, r, q, partials,
                               counter, sc); break;
    case 2: hipLaunchKernelGGL(k_pcg_upd<2>, dim3(nblk_upd), dim3(kKB), 0, st, d, nblk_upd, y, pnew, r, q, partials,
                               counter, sc); break;
    default: hipLaunchKernelGGL(k_pcg_upd<1>, dim3(nblk_upd), dim3(kKB), 0, st, d, nblk_upd, y, pnew, r, q, partials,
                                counter, sc); break;
    }
    if (ev) (void)hipEventRecord(ev[2], st);
}

// One preconditioned CG iteration: z = M^-1 r (and beta), p = z + beta p_old, q = A^ p,
// alpha; y, r update and r.r.
void launch_pcg_line_iter(const Dims &d, int nblk, int nblk_upd, const double *a, const double *lc, const double *lim,
                          double *y, double *r, double *z, double *pold, double *pnew, double *q, double *partials,
                          unsigned *counter, DevScalars *sc, int restart, hipStream_t st, const hipEvent_t *ev)
{
    if (ev) (void)hipEventRecord(ev[0], st);
    hipLaunchKernelGGL(k_line_solve, dim3(nblk), dim3(kKB), 0, st, d, nblk, a, lc, lim, r, z, partials, counter, sc,
                       restart);
    if (ev) (void)hipEventRecord(ev[3], st);
    launch_pcg_dir_upd(d, nblk, nblk_upd, a, z, y, r, pold, pnew, q, partials, counter, sc, st, ev);
}

// ---------------------------------------------------------------- GMRES(m)

// Partial inner products of w with the k basis vectors V_i = V + i n (k <= kMaxBasis),
// eight per pass over the block's cells: partials[blockIdx.x * kMaxBasis + i].
constexpr int kDotGroup = 8;

__global__ __launch_bounds__(kKB) void k_mdot(Dims d, int nblk, const double *__restrict__ V, int k,
                                              const double *__restrict__ w, double *__restrict__ partials)
{
    __shared__ double sh[kKB / 64];
    for (int g0 = 0; g0 < k; g0 += kDotGroup) {
        double acc[kDotGroup];
#pragma unroll
        for (int u = 0; u < kDotGroup; u++) acc[u] = 0.0;
        for_segments<1>(d, nblk, [&](const Row &rw, int i) {
            const long c = rw.base + i;
            const double wv = w[c];
#pragma unroll
            for (int u = 0; u < kDotGroup; u++)
                if (g0 + u < k) acc[u] += V[(long)(g0 + u) * d.n + c] * wv;
        });
#pragma unroll
        for (int u = 0; u < kDotGroup; u++) {
            const double bs = block_sum(acc[u], sh);
            if (threadIdx.x == 0 && g0 + u < k) partials[(long)blockIdx.x * kMaxBasis + g0 + u] = bs;
        }
    }
}

// out[i] = sum over blocks b (in order) of partials[b * kMaxBasis + i]; one block per i.
__global__ __launch_bounds__(kKB) void k_sum_cols(int nblk, const double *__restrict__ partials,
                                                  double *__restrict__ out)
{
    __shared__ double sh[kKB / 64];
    double a = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kKB) a += partials[(long)b * kMaxBasis + blockIdx.x];
    a = block_sum(a, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = a;
}

// w += sign * sum_i coef[i] V_i (coef on the device, i < k, ascending i).
__global__ __launch_bounds__(kKB) void k_maxpy(long n, const double *__restrict__ V, int k,
                                               const double *__restrict__ coef, double sign, double *__restrict__ w)
{
    const long c = (long)blockIdx.x * kKB + threadIdx.x;
    if (c >= n) return;
    double t = 0.0;
    for (int i = 0; i < k; i++) t = fma(coef[i], V[(long)i * n + c], t);
    w[c] = fma(sign, t, w[c]);
}

// y = s x.
__global__ __launch_bounds__(kKB) void k_scale_into(long n, const double *__restrict__ x, double s,
                                                    double *__restrict__ y)
{
    const long c = (long)blockIdx.x * kKB + threadIdx.x;
    if (c < n) y[c] = s * x[c];
}

// y = float(x), and y = double(x): the basis vector a flexible GMRES hands to the network
// (whose input and output are float32) and the network's answer taken back.
__global__ __launch_bounds__(kKB) void k_d2f(long n, const double *__restrict__ x, float *__restrict__ y)
{
    const long c = (long)blockIdx.x * kKB + threadIdx.x;
    if (c < n) y[c] = (float)x[c];
}

__global__ __launch_bounds__(kKB) void k_f2d(long n, const float *__restrict__ x, double *__restrict__ y)
{
    const long c = (long)blockIdx.x * kKB + threadIdx.x;
    if (c < n) y[c] = (double)x[c];
}

void launch_d2f(long n, const double *x, float *y, hipStream_t st)
{
    hipLaunchKernelGGL(k_d2f, dim3((unsigned)((n + kKB - 1) / kKB)), dim3(kKB), 0, st, n, x, y);
}

void launch_f2d(long n, const float *x, double *y, hipStream_t st)
{
    hipLaunchKernelGGL(k_f2d, dim3((unsigned)((n + kKB - 1) / kKB)), dim3(kKB), 0, st, n, x, y);
}

void launch_mdot(const Dims &d, int nblk, const double *V, int k, const double *w, double *partials, double *out,
                 hipStream_t st)
{
    hipLaunchKernelGGL(k_mdot, dim3(nblk), dim3(kKB), 0, st, d, nblk, V, k, w, partials);
    hipLaunchKernelGGL(k_sum_cols, dim3(k), dim3(kKB), 0, st, nblk, partials, out);
}

void launch_maxpy(long n, const double *V, int k, const double *coef, double sign, double *w, hipStream_t st)
{
    hipLaunchKernelGGL(k_maxpy, dim3((unsigned)((n + kKB - 1) / kKB)), dim3(kKB), 0, st, n, V, k, coef, sign, w);
}

void launch_scale_into(long n, const double *x, double s, double *y, hipStream_t st)
{
    hipLaunchKernelGGL(k_scale_into, dim3((unsigned)((n + kKB - 1) / kKB)), dim3(kKB), 0, st, n, x, s, y);
}

}  // namespace rt
