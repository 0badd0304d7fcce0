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
// (4 with the face flux) the wavefront transposes and sums them over bins, and the
// lane that owns each cell (below) scales its sum and stores it, so q, S and the face
// flux leave as coalesced r-contiguous stores.
//
// The opacity table sits in LDS in rows of 64 bins whatever the bin count, so the two
// nodes of a cell are one ds_read2 apart.  The column is read in segments of 512 cells
// (256 with the face flux): lane l owns cells l, l + 64, ... of the segment, loads
// their T and rho with coalesced loads and keeps their table row, (1 - w) rho dr,
// w rho dr and the factors q / sum and S / q.  As the wavefront reaches a cell it takes
// the cell's table row by readlane and its two weights from a per-wave LDS copy of the
// current 64 cells (one broadcast read; the face-flux variants use readlane for these
// too), one cell ahead, so the LDS latency overlaps the current cell's arithmetic.
#include "rt_internal.h"

namespace rt {

constexpr int kWavesPerBlock = 16;  // columns per block
constexpr int kRed = 8;             // sums per transpose (8 lanes add each one)
constexpr int kRowPad = 72;         // LDS doubles per sum row: 64 lanes + 8, so the
                                    // eight rows read together fall in different banks
constexpr int kTabRow = 64;         // LDS doubles per opacity-table row

// Per-cell quantities of a segment, held by the lane that owns the cell (cell
// seg0 + lane + 64 s in slot s): table row offset, the interpolation weights times
// rho dr (floored), q / (sum over bins) = 3 / shell volume and S / q = dr / (rho dr c).
struct CellSlot {
    int kofs;
    double vr, wr, qs, sq;
};

// Sum with the value of lane ^ X (X = 1, 2, 4): ds_swizzle in bit-mask mode (and 0x1f,
// xor X), two 32-bit halves.
template <int X>
__device__ __forceinline__ double add_xor(double v)
{
    int2 t = *reinterpret_cast<int2 *>(&v);
    t.x = __builtin_amdgcn_ds_swizzle(t.x, 0x1f | (X << 10));
    t.y = __builtin_amdgcn_ds_swizzle(t.y, 0x1f | (X << 10));
    return v + *reinterpret_cast<double *>(&t);
}

// v of the lane whose byte address (4 x lane) is addr.
__device__ __forceinline__ double bpermute_d(int addr, double v)
{
    int2 t = *reinterpret_cast<int2 *>(&v);
    t.x = __builtin_amdgcn_ds_bpermute(addr, t.x);
    t.y = __builtin_amdgcn_ds_bpermute(addr, t.y);
    return *reinterpret_cast<double *>(&t);
}

// LDS layout, in doubles: [stage: kWavesPerBlock x 64 x 2, without the face flux]
// [table: nT x kTabRow] [T nodes: nT] [sum rows: kWavesPerBlock x kRed x kRowPad]
// [1 / r_f^2: nr, with the face flux].  The stage leads so its 16-byte pairs are aligned.
__host__ __device__ constexpr size_t stage_doubles(bool face) { return face ? 0 : (size_t)kWavesPerBlock * 128; }

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
    constexpr int kSlots = kFace ? 4 : 8;            // cells per lane in one segment
    constexpr int kSeg = 64 * kSlots;
    constexpr bool kStage = !kFace;                  // weights by LDS broadcast
    extern __shared__ double lds[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double2 *stage = reinterpret_cast<double2 *>(lds) + wave * 64;  // [64] (vr, wr), kStage
    double *tab = lds + stage_doubles(kFace);        // [nT][kTabRow], bins >= nnu zero
    double *Tt = tab + nT * kTabRow;                 // [nT]
    double *red = Tt + nT + wave * (kRed * kRowPad); // [kRed][kRowPad] for this wave
    double *g_f = Tt + nT + kWavesPerBlock * kRed * kRowPad;  // [nr], kFace

    for (int t = threadIdx.x; t < nT * kTabRow; t += blockDim.x) {
        const int k = t / kTabRow, b = t % kTabRow;
        tab[t] = b < nnu ? kap_g[k * nnu + b] : 0.0;
    }
    for (int t = threadIdx.x; t < nT; t += blockDim.x) Tt[t] = Ttab[t];
    if (kFace)
        for (int t = threadIdx.x; t < nr; t += blockDim.x) g_f[t] = 1.0 / rf2[t + 1];
    __syncthreads();

    const long col = (long)blockIdx.x * kWavesPerBlock + wave;
    if (col >= ncol) return;  // no block-wide barrier below this point
    const bool active = lane < nnu;
    const long cbase = col * nr;
    const long fbase = col * (nr + 1);

    double Phi = active ? F0[lane] * R2 : 0.0;
    if (kFace || kBins) {  // face 0 (inner radial boundary): tau = 0
        double v = Phi;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (kFace && lane == 0 && Fface) Fface[fbase] = v / rf2[0];
        if (kBins && active) Fnu[fbase * nnu + lane] = Phi / rf2[0];
    }

    // transpose roles: lane reads sum row `row` at bins part, part + 8, ...; the eight
    // lanes of a row then add across (xor 1, 2, 4), and lane l0 + j takes row j's sum
    const int row = lane >> 3, part = lane & 7;
    const double *rd_lds = red + row * kRowPad + part;
    const double *tab_l = tab + lane;  // this lane's bin in every table row
    for (int seg0 = 0; seg0 < nr; seg0 += kSeg) {
        CellSlot cs[kSlots];
#pragma unroll
        for (int sl = 0; sl < kSlots; sl++) {
            const int i = seg0 + lane + 64 * sl;
            const int ic = i < nr ? i : nr - 1;
            const long c = cbase + ic;
            const double t = T[c], rh = rho[c], d = dr[ic], sh = shell[ic];
            int k;
            double w;
            lin_node(Tt, nT, t, k, w);
            const double v = rh * d;
            const double rdr = v > 1e-250 ? v : 1e-250;  // keeps S = q / (rho c) finite as rho -> 0
            cs[sl].kofs = k * kTabRow;
            cs[sl].vr = (1.0 - w) * rdr;
            cs[sl].wr = w * rdr;
            cs[sl].qs = 3.0 / sh;
            cs[sl].sq = d / (rdr * kC);
        }
#pragma unroll
        for (int sl = 0; sl < kSlots; sl++) {
            const int sbase = seg0 + 64 * sl;
            if (sbase >= nr) break;
            if (kStage) {  // this slot's weights to the wave's stage (earlier reads are done)
                wave_sync();
                stage[lane] = make_double2(cs[sl].vr, cs[sl].wr);
                wave_sync();
            }
            // table entries and weights of cell l of the slot
            double a0, a1, vr, wr;
            auto fetch = [&](int l) {
                const int ko = __builtin_amdgcn_readlane(cs[sl].kofs, l);
                a0 = tab_l[ko];
                a1 = tab_l[ko + kTabRow];
                if (kStage) {
                    const double2 p = stage[l];
                    vr = p.x;
                    wr = p.y;
                } else {
                    vr = readlane_d(cs[sl].vr, l);
                    wr = readlane_d(cs[sl].wr, l);
                }
            };
            fetch(0);
            for (int l0 = 0; l0 < 64; l0 += kChunk) {
                const int i0 = sbase + l0;
                if (i0 >= nr) break;
                const int ncell = (nr - i0) < kChunk ? (nr - i0) : kChunk;
#pragma unroll
                for (int m = 0; m < kChunk; m++) {
                    if (m < ncell) {
                        const double dtau = fma(wr, a1, vr * a0);
                        // the next cell's (after the slot's last cell, lane 0's again: in
                        // range, and the next slot fetches afresh)
                        fetch((l0 + m + 1) & 63);
                        double e, em;
                        exp_pair(dtau, e, em);
                        red[m * kRowPad + lane] = Phi * em;   // absorbed, before the 3/shell factor
                        Phi = Phi * e;
                        if (kFace) red[(kChunk + m) * kRowPad + lane] = Phi;  // through the outer face
                        // per-bin flux at that face: one 64-bin row per face, bin fastest
                        if (kBins && active) Fnu[(fbase + i0 + m + 1) * nnu + lane] = Phi * g_f[i0 + m];
                    }
                }
                wave_sync();
                double acc = rd_lds[0];
#pragma unroll
                for (int t = 1; t < 8; t++) acc += rd_lds[8 * t];
                acc = add_xor<1>(acc);
                acc = add_xor<2>(acc);
                acc = add_xor<4>(acc);
                // row j's sum to lane (l0 + j) mod 64: cells j < kChunk land on their
                // owners; with the face flux, the faces' rows follow them, wrapping to
                // lanes 0-3 after the slot's last chunk (with 8-cell chunks l0 is a
                // multiple of 8 and j = lane & 7)
                const int j = (lane - l0) & 63;
                acc = bpermute_d(32 * (kFace ? (j & 7) : (lane & 7)), acc);
                wave_sync();
                if ((unsigned)j < (unsigned)ncell) {  // the owner of cell i0 + j
                    const int i = sbase + lane;         // = i0 + j
                    const double qv = cs[sl].qs * acc;
                    q[cbase + i] = qv;
                    S[cbase + i] = qv * cs[sl].sq;
                } else if (kFace && Fface && (unsigned)(j - kChunk) < (unsigned)ncell) {
                    const int i = i0 + j - kChunk;
                    Fface[fbase + i + 1] = acc * g_f[i];
                }
            }
        }
    }
}

void launch_raytrace_bins(const Dims &d, const Opac &op, const Geo &g, const double *F0, double R2,
                          const double *rho, const double *T, double *q, double *S, double *Fface,
                          double *Fnu, hipStream_t st)
{
    long ncol = (long)d.nt * d.np;
    long nblk = (ncol + kWavesPerBlock - 1) / kWavesPerBlock;
    const bool face = Fnu || Fface;
    size_t lds = raytrace_lds_bytes(op.nT, d.nr, face);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(64 * kWavesPerBlock), lds, st, d.nr, ncol, op.nnu, op.nT,
                           rho, T, op.T, op.kap, F0, R2, g.rf2, g.dr, g.shell, q, S, Fface, Fnu);
    };
    if (Fnu) go(k_raytrace<true, true>);
    else if (Fface) go(k_raytrace<true, false>);
    else go(k_raytrace<false, false>);
}

// q and S alone: lanes on cells where the column fills its 512-cell segments to 90 % or
// more (measured faster there: fewer instructions per cell and bin, no transpose), else
// lanes on bins; the face fluxes always come from lanes on bins.
void launch_raytrace(const Dims &d, const Opac &op, const Geo &g, const double *F0, double R2,
                     const double *rho, const double *T, double *q, double *S, double *Fface,
                     double *Fnu, hipStream_t st)
{
    if (!Fface && !Fnu && raytrace_cells_fit(d.nr)) launch_raytrace_r(d, op, g, F0, R2, rho, T, q, S, st);
    else launch_raytrace_bins(d, op, g, F0, R2, rho, T, q, S, Fface, Fnu, st);
}

void raytrace_prepare()
{
    // the whole LDS of a compute unit, so contexts with any column length can launch
    for (const void *k : {(const void *)k_raytrace<false, false>, (const void *)k_raytrace<true, false>,
                          (const void *)k_raytrace<true, true>})
        (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    raytrace_r_prepare();
}

size_t raytrace_lds_bytes(int nT, int nr, bool face)
{
    return sizeof(double) * (stage_doubles(face) + (size_t)nT * kTabRow + nT +
                             (size_t)kWavesPerBlock * kRed * kRowPad + (face ? (size_t)nr : 0));
}

}  // namespace rt
