// The ray trace with the other mapping of a radial column onto a wavefront: lanes on
// radial cells instead of frequency bins (Kuiper et al., Sect. "Irradiation", Eqs. 17
// and 19; Sect. "Frequency dependent irradiation", Eq. 20; cell-integrated absorption
// of Eqs. 28-36).  It computes the same q_star and S_abs as k_raytrace, to rounding
// order; measured on gfx950 it is the faster of the two where a column fills its
// 512-cell segments (27.6 instead of 31.3 float64 instructions per cell and bin: no
// transpose for the bin sums, one LDS read per cell and bin), so the step's ray trace
// uses it there.
//
// One wavefront per radial column (j, k); the column is taken in segments of 512 cells,
// lane l owning the 8 consecutive cells 8 l .. 8 l + 7 of a segment.  For each bin b in
// turn every lane forms its cells' transmissions e = exp(-dtau_b) and absorptions
// 1 - e (exp_pair), their running product inside the lane, and the product over the
// lanes before it by a multiplicative scan across the wavefront (DPP row shifts and row
// broadcasts); the flux entering cell i is then the bin's flux at the segment's inner
// face times these two products, and the cell's absorbed power of bin b is added to its
// own register (the sum over bins never leaves the lane).  The flux carried from one
// segment to the next sits in lane b of one register.
//
// The opacity table is in LDS bin-major, [bin][T node], so a cell's two interpolation
// nodes are one ds_read2 apart, and the neighbouring cells of a column (nearby
// temperatures) read the same or nearby words.
#include <type_traits>

#include "rt_internal.h"

namespace rt {

constexpr int kRCells = 8;                 // cells per lane in a segment
constexpr int kRSeg = 64 * kRCells;        // cells per segment
constexpr int kRWaves = 8;                 // columns per block

// One step of the inclusive multiplicative scan across the wavefront: v times the value
// the DPP control CTRL moves into this lane (1 where it moves none, or outside ROWS).
template <int CTRL, int ROWS>
__device__ __forceinline__ double scan_mul_step(double v)
{
    int2 t = *reinterpret_cast<int2 *>(&v);
    t.x = __builtin_amdgcn_update_dpp(0, t.x, CTRL, ROWS, 0xf, false);
    t.y = __builtin_amdgcn_update_dpp(0x3FF00000, t.y, CTRL, ROWS, 0xf, false);  // 1.0
    return v * *reinterpret_cast<double *>(&t);
}

// Product of v over the lanes below this one (1 in lane 0).
__device__ __forceinline__ double exclusive_scan_mul(double v)
{
    {  // shift up by one lane (wave_shr:1), lane 0 takes 1
        int2 t = *reinterpret_cast<int2 *>(&v);
        t.x = __builtin_amdgcn_update_dpp(0, t.x, 0x138, 0xf, 0xf, false);
        t.y = __builtin_amdgcn_update_dpp(0x3FF00000, t.y, 0x138, 0xf, 0xf, false);
        v = *reinterpret_cast<double *>(&t);
    }
    v = scan_mul_step<0x111, 0xf>(v);  // row_shr:1
    v = scan_mul_step<0x112, 0xf>(v);  // row_shr:2
    v = scan_mul_step<0x114, 0xf>(v);  // row_shr:4
    v = scan_mul_step<0x118, 0xf>(v);  // row_shr:8: each row of 16 lanes scanned
    v = scan_mul_step<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v = scan_mul_step<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

__global__ __launch_bounds__(64 * kRWaves) void k_raytrace_r(
    int nr, long ncol, int nnu, int nT, int kconst,
    const double *__restrict__ rho, const double *__restrict__ T,
    const double *__restrict__ Ttab, const double *__restrict__ kap_g,
    const double *__restrict__ F0, double R2,
    const double *__restrict__ dr, const double *__restrict__ shell,
    double *__restrict__ q, double *__restrict__ S)
{
    extern __shared__ double lds[];
    double *tab = lds;              // [nnu][nT]
    double *Tt = tab + nnu * nT;    // [nT]
    for (int t = threadIdx.x; t < nnu * nT; t += blockDim.x) {
        const int b = t / nT, k = t - b * nT;
        tab[t] = kap_g[k * nnu + b];
    }
    for (int t = threadIdx.x; t < nT; t += blockDim.x) Tt[t] = Ttab[t];
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const long col = (long)blockIdx.x * kRWaves + (threadIdx.x >> 6);
    if (col >= ncol) return;  // no block-wide barrier below this point
    const long cbase = col * nr;
    // lane b: the flux of bin b at the current segment's inner face (times r^2)
    double carry = lane < nnu ? F0[lane] * R2 : 0.0;

    for (int seg0 = 0; seg0 < nr; seg0 += kRSeg) {
        const int i0 = seg0 + kRCells * lane;  // this lane's first cell
        // per cell: table node k and weight w, rho dr (floored); vr / wr hold rho dr and w
        // until the wavefront knows whether all its cells lie in the T-independent rows
        int kofs[kRCells];
        double vr[kRCells], wr[kRCells], acc[kRCells];
        bool cold = true;  // every node this lane's cells use is a T-independent row
#pragma unroll
        for (int s = 0; s < kRCells; s++) {
            acc[s] = 0.0;
            const int i = i0 + s;
            if (i < nr) {
                const double t = T[cbase + i], v = rho[cbase + i] * dr[i];
                int k;
                double w;
                lin_node(Tt, nT, t, k, w);
                kofs[s] = k;
                vr[s] = v > 1e-250 ? v : 1e-250;
                wr[s] = w;
                cold = cold && k + 1 < kconst;
            } else {  // beyond the column: transmission 1, nothing absorbed
                kofs[s] = 0;
                vr[s] = wr[s] = 0.0;
            }
        }
        // Below sublimation kappa_nu does not depend on T: where the whole wavefront's
        // cells use only such rows, dtau = kappa_nu (row 0) x rho dr, one uniform table
        // value per bin; otherwise the interpolation weights (1 - w) rho dr, w rho dr.
        const bool fast = __all(cold);
        if (!fast) {
#pragma unroll
            for (int s = 0; s < kRCells; s++) {
                const double rdr = vr[s], w = wr[s];
                vr[s] = (1.0 - w) * rdr;
                wr[s] = w * rdr;
            }
        }
        const bool last = seg0 + kRSeg >= nr;
        auto bins = [&](auto fc) __attribute__((always_inline)) {
            constexpr bool kFast = decltype(fc)::value;
            for (int b = 0; b < nnu; b++) {
                const double *tb = tab + b * nT;
                const double kb = kFast ? tb[0] : 0.0;
                double P = 1.0, a[kRCells];
#pragma unroll
                for (int s = 0; s < kRCells; s++) {
                    const double dtau = kFast ? kb * vr[s] : fma(wr[s], tb[kofs[s] + 1], vr[s] * tb[kofs[s]]);
                    double e, m;
                    exp_pair(dtau, e, m);
                    a[s] = P * m;  // absorbed fraction of the flux entering this lane's cells
                    P = P * e;
                }
                const double X = exclusive_scan_mul(P);
                const double C = readlane_d(carry, b);
                const double G = C * X;  // flux of bin b entering this lane's first cell
#pragma unroll
                for (int s = 0; s < kRCells; s++) acc[s] = fma(G, a[s], acc[s]);
                if (!last) {  // the bin's flux at the next segment's inner face, into lane b
                    const double through = readlane_d(X * P, 63);
                    if (lane == b) carry = C * through;
                }
            }
        };
        if (fast) bins(std::true_type{});
        else bins(std::false_type{});
#pragma unroll
        for (int s = 0; s < kRCells; s++) {
            const int i = i0 + s;
            if (i < nr) {
                const double v = rho[cbase + i] * dr[i];
                const double rdr = v > 1e-250 ? v : 1e-250;
                const double qv = (3.0 / shell[i]) * acc[s];
                q[cbase + i] = qv;
                S[cbase + i] = qv * (dr[i] / (rdr * kC));
            }
        }
    }
}

size_t raytrace_r_lds_bytes(int nT, int nnu) { return sizeof(double) * ((size_t)nnu * nT + nT); }

bool raytrace_cells_fit(int nr)
{
    const long seg = (nr + kRSeg - 1) / kRSeg;
    return 10L * nr >= 9L * seg * kRSeg;
}

void raytrace_r_prepare()
{
    (void)hipFuncSetAttribute((const void *)k_raytrace_r, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

void launch_raytrace_r(const Dims &d, const Opac &op, const Geo &g, const double *F0, double R2, const double *rho,
                       const double *T, double *q, double *S, hipStream_t st)
{
    const long ncol = (long)d.nt * d.np;
    const long nblk = (ncol + kRWaves - 1) / kRWaves;
    hipLaunchKernelGGL(k_raytrace_r, dim3((unsigned)nblk), dim3(64 * kRWaves), raytrace_r_lds_bytes(op.nT, op.nnu), st,
                       d.nr, ncol, op.nnu, op.nT, op.kconst, rho, T, op.T, op.kap, F0, R2, g.dr, g.shell, q, S);
}

}  // namespace rt
