// Frequency-dependent first-order ray trace of the stellar irradiation along radial
// rays (Kuiper et al., Sect. "Irradiation", Eqs. 17 and 19; Sect. "Frequency
// dependent irradiation", Eq. 20; cell-integrated absorption of Eqs. 28-36).
//
// Mapping: one wavefront per radial column (j, k); lane b owns frequency bin b and
// walks the column outward cell by cell, carrying Phi_b = F_b(R_*) R_*^2 exp(-tau_b)
// in float64 (the optical depth enters as the running product of the cell
// transmissions exp(-dtau), each from one range reduction together with
// 1 - exp(-dtau)).  Per cell, the per-bin absorbed power Phi_b (1 - exp(-dtau_b)) (and,
// when the face flux is asked for, the outgoing Phi_b) is parked in LDS; every 8 cells
// (4 with the face flux) the wavefront transposes and sums them over bins, so q, S and
// the face flux leave as coalesced r-contiguous stores.  The opacity table and the radial geometry factors of the column sit in LDS;
// the column is read in segments of 512 cells, each lane loading T and rho of 8 cells
// with coalesced loads and computing their table node, weight and rho dr, which the
// wavefront broadcasts with readlane as it reaches each cell.
#include "rt_internal.h"

namespace rt {

constexpr int kWavesPerBlock = 16; // columns per block
constexpr int kSlots = 8;          // cells per lane in one segment
constexpr int kSeg = 64 * kSlots;  // cells per segment of a column
constexpr int kRed = 8;            // sums per transpose (8 lanes add each one)

// Per-cell quantities of a segment, held by the lane that owns the cell (cell
// seg0 + lane + 64 s in slot s) and broadcast with readlane when the wavefront reaches
// it: the table row offset and weight, rho dr (floored).
struct CellSlot {
    int kofs;
    double w, rdr;
};

// kFace: also the total flux at every radial face, Fface when not NULL (the transpose
// then sums 4 cells' absorbed power and 4 faces' flux; without it 8 cells' absorbed
// power).  kBins (with kFace): also the per-bin face flux Fnu.  Separate
// instantiations, so the step's ray trace (neither) keeps the shortest schedule.
template <bool kFace, bool kBins>
__global__ __launch_bounds__(1024) void k_raytrace(
    int nr, long ncol, int nnu, int nT,
    const double *__restrict__ rho, const double *__restrict__ T,
    const double *__restrict__ Ttab, const double *__restrict__ kap_g,
    const double *__restrict__ F0, double R2,
    const double *__restrict__ rf2, const double *__restrict__ dr, const double *__restrict__ shell,
    double *__restrict__ q, double *__restrict__ S, double *__restrict__ Fface, double *__restrict__ Fnu)
{
    constexpr int kChunk = kFace ? kRed / 2 : kRed;  // cells per transpose
    extern __shared__ double lds[];
    double *tab = lds;                       // [nT][nnu]
    double *Tt = tab + nT * nnu;             // [nT]
    double *g_dr = Tt + nT;                  // [nr] dr
    double *g_q = g_dr + nr;                 // [nr] 3 / shell volume
    double *g_f = g_q + nr;                  // [nr] 1 / r_f^2 of the outer face
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double *red = g_f + nr + wave * (kRed * 64);  // [kRed][64] for this wave

    for (int t = threadIdx.x; t < nT * nnu; t += blockDim.x) tab[t] = kap_g[t];
    for (int t = threadIdx.x; t < nT; t += blockDim.x) Tt[t] = Ttab[t];
    for (int t = threadIdx.x; t < nr; t += blockDim.x) {
        g_dr[t] = dr[t];
        g_q[t] = 3.0 / shell[t];
        g_f[t] = 1.0 / rf2[t + 1];
    }
    __syncthreads();

    const long col = (long)blockIdx.x * kWavesPerBlock + wave;
    if (col >= ncol) return;  // no block-wide barrier below this point
    const bool active = lane < nnu;
    const int lb = active ? lane : 0;
    const long cbase = col * nr;
    const long fbase = col * (nr + 1);

    double Phi = active ? F0[lane] * R2 : 0.0;
    if (kFace || kBins) {  // face 0 (inner radial boundary): tau = 0
        double v = Phi;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (kFace && lane == 0 && Fface) Fface[fbase] = v / rf2[0];
        if (kBins && active) Fnu[fbase * nnu + lane] = Phi / rf2[0];
    }

    const int s8 = lane >> 3, part = lane & 7;  // reduction roles: sum s8 of kRed, part of 8
    for (int seg0 = 0; seg0 < nr; seg0 += kSeg) {
        // one coalesced batch of loads per segment: slot s holds cell seg0 + lane + 64 s
        CellSlot cs[kSlots];
#pragma unroll
        for (int sl = 0; sl < kSlots; sl++) {
            const int i = seg0 + lane + 64 * sl;
            const bool in = i < nr;
            const int ic = in ? i : nr - 1;
            const long c = cbase + ic;
            const double t = T[c], rh = rho[c];
            int k;
            lin_node(Tt, nT, t, k, cs[sl].w);
            cs[sl].kofs = k * nnu;
            const double v = rh * g_dr[ic];
            cs[sl].rdr = v > 1e-250 ? v : 1e-250;  // keeps S = q / (rho c) finite as rho -> 0
        }
#pragma unroll
        for (int sl = 0; sl < kSlots; sl++) {
            const int sbase = seg0 + 64 * sl;
            if (sbase >= nr) break;
            for (int l0 = 0; l0 < 64; l0 += kChunk) {
                const int i0 = sbase + l0;
                if (i0 >= nr) break;
                const int ncell = (nr - i0) < kChunk ? (nr - i0) : kChunk;
#pragma unroll
                for (int m = 0; m < kChunk; m++) {
                    if (m < ncell) {
                        const int ko = __builtin_amdgcn_readlane(cs[sl].kofs, l0 + m);
                        const double w = readlane_d(cs[sl].w, l0 + m);
                        const double rd = readlane_d(cs[sl].rdr, l0 + m);
                        const double a0 = tab[ko + lb], a1 = tab[ko + nnu + lb];
                        double e, em;
                        exp_pair(fma(w, a1 - a0, a0) * rd, e, em);
                        red[m * 64 + lane] = Phi * em;   // absorbed, before the 3/shell factor
                        Phi = Phi * e;
                        if (kFace) red[(kChunk + m) * 64 + lane] = Phi;  // through the outer face
                        // per-bin flux at that face: one 64-bin row per face, bin fastest
                        if (kBins && active) Fnu[(fbase + i0 + m + 1) * nnu + lane] = Phi * g_f[i0 + m];
                    }
                }
                wave_sync();
                // kRed sums over the 64 lanes: lane -> (sum s8, part), 8 values each
                double acc = 0.0;
#pragma unroll
                for (int t = 0; t < 8; t++) acc += red[s8 * 64 + part + 8 * t];
                acc += __shfl_xor(acc, 1);
                acc += __shfl_xor(acc, 2);
                acc += __shfl_xor(acc, 4);
                // rho dr of the chunk's cells, uniform per cell
                double rd8[kChunk];
#pragma unroll
                for (int m = 0; m < kChunk; m++) rd8[m] = readlane_d(cs[sl].rdr, l0 + m);
                wave_sync();
                if (part == 0) {
                    const int mm = s8 < kChunk ? s8 : s8 - kChunk;
                    const int i = i0 + mm;
                    if (i < nr) {
                        if (s8 < kChunk) {
                            double rdm = rd8[0];
#pragma unroll
                            for (int m = 1; m < kChunk; m++) rdm = mm == m ? rd8[m] : rdm;
                            const double qv = g_q[i] * acc;
                            q[cbase + i] = qv;
                            S[cbase + i] = qv * g_dr[i] / (rdm * kC);
                        } else if (kFace && Fface) {
                            Fface[fbase + i + 1] = acc * g_f[i];
                        }
                    }
                }
            }
        }
    }
}

void launch_raytrace(const Dims &d, const Opac &op, const Geo &g, const double *F0, double R2,
                     const double *rho, const double *T, double *q, double *S, double *Fface,
                     double *Fnu, hipStream_t st)
{
    long ncol = (long)d.nt * d.np;
    long nblk = (ncol + kWavesPerBlock - 1) / kWavesPerBlock;
    size_t lds = raytrace_lds_bytes(op.nT, op.nnu, d.nr);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(64 * kWavesPerBlock), lds, st, d.nr, ncol, op.nnu, op.nT,
                           rho, T, op.T, op.kap, F0, R2, g.rf2, g.dr, g.shell, q, S, Fface, Fnu);
    };
    if (Fnu) go(k_raytrace<true, true>);
    else if (Fface) go(k_raytrace<true, false>);
    else go(k_raytrace<false, false>);
}

void raytrace_prepare(size_t lds_bytes)
{
    for (const void *k : {(const void *)k_raytrace<false, false>, (const void *)k_raytrace<true, false>,
                          (const void *)k_raytrace<true, true>})
        (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

size_t raytrace_lds_bytes(int nT, int nnu, int nr)
{
    return sizeof(double) * ((size_t)nT * nnu + nT + 3 * (size_t)nr + (size_t)kWavesPerBlock * kRed * 64);
}

}  // namespace rt
