// Frequency-dependent first-order ray trace of the stellar irradiation along radial
// rays (Kuiper et al., Sect. "Irradiation", Eqs. 17 and 19; Sect. "Frequency
// dependent irradiation", Eq. 20; cell-integrated absorption of Eqs. 28-36).
//
// Mapping: one wavefront per radial column (j, k); lane b owns frequency bin b and
// walks the column outward cell by cell, carrying Phi_b = F_b(R_*) R_*^2 exp(-tau_b)
// in float64 (the optical depth enters as the running product of the cell
// transmissions exp(-dtau), each from one range reduction together with
// 1 - exp(-dtau)).  Per cell, the per-bin absorbed power Phi_b (1 - exp(-dtau_b)) and
// the outgoing Phi_b are parked in LDS; every kChunk cells the wavefront transposes
// and sums them over bins, so q, S and the face flux leave as coalesced r-contiguous
// stores.  The opacity table sits in LDS; per-cell table coordinates are computed by
// kChunk lanes and broadcast with readlane.
#include "rt_internal.h"

namespace rt {

constexpr int kChunk = 4;          // cells per transpose
constexpr int kWavesPerBlock = 16; // columns per block

__global__ __launch_bounds__(1024) void k_raytrace(
    int nr, long ncol, int nnu, int nT,
    const double *__restrict__ rho, const double *__restrict__ T,
    const double *__restrict__ Ttab, const double *__restrict__ kap_g,
    const double *__restrict__ F0, double R2,
    const double *__restrict__ rf2, const double *__restrict__ dr, const double *__restrict__ shell,
    double *__restrict__ q, double *__restrict__ S, double *__restrict__ Fface)
{
    extern __shared__ double lds[];
    double *tab = lds;                       // [nT][nnu]
    double *Tt = tab + nT * nnu;             // [nT]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double *red = Tt + nT + wave * (2 * kChunk * 64);  // [2][kChunk][64] for this wave

    for (int t = threadIdx.x; t < nT * nnu; t += blockDim.x) tab[t] = kap_g[t];
    for (int t = threadIdx.x; t < nT; t += blockDim.x) Tt[t] = Ttab[t];
    __syncthreads();

    const long col = (long)blockIdx.x * kWavesPerBlock + wave;
    if (col >= ncol) return;  // no block-wide barrier below this point
    const bool active = lane < nnu;
    const int lb = active ? lane : 0;
    const long cbase = col * nr;
    const long fbase = col * (nr + 1);

    double Phi = active ? F0[lane] * R2 : 0.0;
    {   // face 0 (inner radial boundary): tau = 0
        double v = Phi;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0 && Fface) Fface[fbase] = v / rf2[0];
    }

    for (int i0 = 0; i0 < nr; i0 += kChunk) {
        // table coordinates and rho*dr of the chunk's cells, one lane per cell
        int kk = 0;
        double ww = 0.0, rdr = 1e-250, rh = 0.0;
        if (lane < kChunk && i0 + lane < nr) {
            long c = cbase + i0 + lane;
            double t = T[c];
            rh = rho[c];
            lin_node(Tt, nT, t, kk, ww);
            double v = rh * dr[i0 + lane];
            rdr = v > 1e-250 ? v : 1e-250;  // keeps S = q / (rho c) finite as rho -> 0
        }
        const int ncell = (nr - i0) < kChunk ? (nr - i0) : kChunk;
#pragma unroll
        for (int m = 0; m < kChunk; m++) {
            if (m < ncell) {
                int k = __builtin_amdgcn_readlane(kk, m);
                double w = readlane_d(ww, m);
                double rd = readlane_d(rdr, m);
                double a0 = tab[k * nnu + lb], a1 = tab[(k + 1) * nnu + lb];
                double kap = (1.0 - w) * a0 + w * a1;
                double e, em;
                exp_pair(kap * rd, e, em);
                red[m * 64 + lane] = Phi * em;   // absorbed, before the 3/shell factor
                Phi = Phi * e;
                red[(kChunk + m) * 64 + lane] = Phi;  // through the outer face
            }
        }
        wave_sync();
        // 2*kChunk sums over the 64 lanes: lane -> (sum s, part), 8 values each
        const int s = lane >> 3, part = lane & 7;
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < 8; t++) acc += red[s * 64 + part + 8 * t];
        acc += __shfl_xor(acc, 1);
        acc += __shfl_xor(acc, 2);
        acc += __shfl_xor(acc, 4);
        wave_sync();
        if (part == 0) {
            if (s < kChunk) {
                int i = i0 + s;
                if (i < nr) {
                    long c = cbase + i;
                    double qv = 3.0 * acc / shell[i];
                    q[c] = qv;
                    double rdr_c = rho[c] * dr[i];
                    rdr_c = rdr_c > 1e-250 ? rdr_c : 1e-250;
                    S[c] = qv * dr[i] / (rdr_c * kC);
                }
            } else {
                int i = i0 + (s - kChunk);
                if (i < nr && Fface) Fface[fbase + i + 1] = acc / rf2[i + 1];
            }
        }
        (void)rh;
    }
}

void launch_raytrace(const Dims &d, const Opac &op, const Geo &g, const double *F0, double R2,
                     const double *rho, const double *T, double *q, double *S, double *Fface,
                     hipStream_t st)
{
    long ncol = (long)d.nt * d.np;
    long nblk = (ncol + kWavesPerBlock - 1) / kWavesPerBlock;
    size_t lds = sizeof(double) * ((size_t)op.nT * op.nnu + op.nT + (size_t)kWavesPerBlock * 2 * kChunk * 64);
    hipLaunchKernelGGL(k_raytrace, dim3((unsigned)nblk), dim3(64 * kWavesPerBlock), lds, st,
                       d.nr, ncol, op.nnu, op.nT, rho, T, op.T, op.kap, F0, R2, g.rf2, g.dr, g.shell,
                       q, S, Fface);
}

void raytrace_prepare(size_t lds_bytes)
{
    (void)hipFuncSetAttribute((const void *)k_raytrace, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

size_t raytrace_lds_bytes(int nT, int nnu)
{
    return sizeof(double) * ((size_t)nT * nnu + nT + (size_t)kWavesPerBlock * 2 * kChunk * 64);
}

}  // namespace rt
