// Kernels of the learned preconditioner: a 3-level 3-D convolutional U-Net (3x3x3
// kernels, 16/32/64 channels) evaluated and trained in BF16 on the matrix cores with
// FP32 accumulation.
//
// Tensors are channels-last, x[c * C + ch], on the spherical grid levels (cell
// c = i + nr (j + nt k)); convolutions pad with zeros in r and theta and wrap in phi.
// Tap t = (dk+1) 9 + (dj+1) 3 + (di+1); weights w[(t Cout + co) Cin + ci] (and a
// transposed copy wt[(t Cin + ci) Cout + co] for the data gradient).
//
// Every 3x3x3 convolution (forward and data gradient) is an LDS-tiled implicit GEMM on
// v_mfma_f32_16x16x32_bf16 with the weights as A and the activations as B: M = 16
// output channels of one output-channel tile, N = 16 cells of a radial row segment,
// K = 32 = two taps x 16 input channels of one input slice.  Lane l supplies
// A[m = l%16][k = 8(l/16) .. +7] (8 input channels of one tap for output channel l%16,
// staged in LDS in this fragment order) and B[k = 8(l/16) .. +7][n = l%16] (8 channels
// of cell l%16's neighbour through that tap, from the LDS tile), and receives
// D[m = 4(l/16) .. +3][n = l%16]: 4 consecutive output channels of one cell, stored as
// one vector (conv_tiles below).  The weight gradient is its own MFMA kernel
// (k_conv_wgrad: M = output channels, N = input channels, K = 32 cells of a radial
// row).  A decoder convolution reads two sources (the nearest-neighbour upsampled
// coarse tensor and the skip tensor) directly, so the upsampled / concatenated tensor
// is never materialised.
#include <type_traits>

#include "rt_internal.h"

namespace rt {
namespace nn {

typedef unsigned short bf16;
typedef short short4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));

constexpr int kTB = 256;

__device__ __forceinline__ float bf2f(bf16 h) { return __uint_as_float((unsigned)h << 16); }
// Round to nearest even; NaN stays a quiet NaN.
__device__ __forceinline__ bf16 f2bf(float f)
{
    unsigned u = __float_as_uint(f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (bf16)0x7FC0u;
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (bf16)(u >> 16);
}

// Four bf16 at p (8-byte aligned) as an MFMA operand, or zeros when !ok.
__device__ __forceinline__ short4v ld4(const bf16 *__restrict__ p, bool ok)
{
    uint2 u = *reinterpret_cast<const uint2 *>(p);
    short4v v = *reinterpret_cast<short4v *>(&u);
    short4v z = {0, 0, 0, 0};
    return ok ? v : z;
}

// Four fp32 gradients at p, masked by the ReLU output y > 0 (when y != nullptr) and
// rounded to bf16 as an MFMA operand; zeros when !ok.
__device__ __forceinline__ short4v ld4_grad(const float *__restrict__ g, const bf16 *__restrict__ y, bool ok)
{
    float4 v = *reinterpret_cast<const float4 *>(g);
    float f[4] = {v.x, v.y, v.z, v.w};
    if (y) {
        uint2 u = *reinterpret_cast<const uint2 *>(y);
        const bf16 *h = reinterpret_cast<const bf16 *>(&u);
#pragma unroll
        for (int q = 0; q < 4; q++)
            if (!(bf2f(h[q]) > 0.0f)) f[q] = 0.0f;
    }
    short4v o;
#pragma unroll
    for (int q = 0; q < 4; q++) o[q] = ok ? (short)f2bf(f[q]) : (short)0;
    return o;
}

__device__ __forceinline__ void cell_coords(const Lv &L, long c, int &i, int &j, int &k)
{
    i = (int)(c % L.nr);
    long jk = c / L.nr;
    j = (int)(jk % L.nt);
    k = (int)(jk / L.nt);
}

// Neighbour of (i, j, k) through tap t (sign = +1) or its mirror (sign = -1).
__device__ __forceinline__ bool tap_nb(const Lv &L, int i, int j, int k, int t, int sign, int &a, int &b, int &c)
{
    a = i + sign * (t % 3 - 1);
    b = j + sign * ((t / 3) % 3 - 1);
    c = k + sign * (t / 9 - 1);
    c = c < 0 ? c + L.np : (c >= L.np ? c - L.np : c);
    return (unsigned)a < (unsigned)L.nr && (unsigned)b < (unsigned)L.nt;
}

// Compile-time loop: f(std::integral_constant<int, i>{}) for i = B .. E-1.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// ------------------------------------------------------ tiled convolution

// Forward and data-gradient convolutions share one LDS-tiled implicit GEMM.  A block
// owns kTR x TJ x TK output cells (r x theta x phi).  For each 16-channel input slice
// it stages the input tile with a one-cell halo (zeros outside r and theta, wrapped in
// phi) and the slice's weights of all 27 taps in LDS, then runs
// v_mfma_f32_16x16x32_bf16 with K = two taps x 16 channels:
//   A[m = output channel][k] = weights, lane l holding 8 channels of tap 2p + l/32 for
//     output channel l%16 (stored in LDS in exactly this fragment order; a 28th tap of
//     zeros pads the last pair);
//   B[k][n = cell] = activations, lane l holding 8 channels of the neighbour, through
//     the same tap, of cell l%16 of a 16-cell row segment;
//   D[m = 4(l/16) + i][n = l%16]: each lane ends with 4 consecutive output channels of
//     one cell, stored as one vector.
// Each wavefront owns Tile::per_wave row segments (adjacent in r and theta), so one A
// fragment feeds that many MFMAs and one B fragment feeds NT output-channel tiles.
// The LDS tile is stored cell-major, xs[cell][h][8] with h the lower or upper 8
// channels (32 bytes per cell), so the 32 lanes of one tap in a fragment read 512
// contiguous bytes and the other tap's 32 lanes another 512; measured on gfx950 this is
// free of bank conflicts for every tap distance, where a half-major layout (halves a
// tile apart) costs every fragment read a second pass.  The tile is written with
// contiguous 16-byte stores, and every fragment address is a per-lane base plus a
// compile-time offset for the segment and the tap.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));

constexpr int kTR = 32;

template <int TJ, int TK>
struct Tile {
    static constexpr int HR = kTR + 2, HJ = TJ + 2, HK = TK + 2;
    static constexpr int cells = HR * HJ * HK;
    static constexpr int segs = 2 * TJ * TK;  // 16-cell row segments
    static constexpr int per_wave = segs / 4;
    static_assert(per_wave % 2 == 0 && (2 * TJ) % per_wave == 0, "a wavefront's segments share one phi plane");
};

// LDS bytes of one block: input tile of one slice plus the slice's weights (28 taps).
template <int NT, int TJ, int TK>
constexpr size_t conv_lds_bytes() { return (size_t)Tile<TJ, TK>::cells * 32 + 28 * NT * 512; }

// Two floats to two bf16 (round to nearest even, NaN stays NaN) packed in 32 bits.
__device__ __forceinline__ unsigned pack_bf16(float a, float b)
{
    const bf16x2 h = __builtin_convertvector(float2v{a, b}, bf16x2);
    return *reinterpret_cast<const unsigned *>(&h);
}

// Body shared by the forward (sign = +1) and data-gradient (sign = -1: the output cell
// whose tap reads this cell) convolutions.  load(idx, a, b, c, ch) issues the loads of
// 8 input channels ch .. ch + 7 of cell idx = (a, b, c) (cell 0 for cells outside the
// grid, so every address is valid) and returns them raw; finish(raw, ok) turns them
// into 8 bf16 operands, zeros where !ok, when the tile is written to LDS (so a load
// issued ahead is not waited for early); store(idx, ch, v) writes output channels
// ch .. ch + 3.  w is [tap][cout][cin] in bf16.  AHEAD: the next item's tile and
// weights are loaded before this item's MFMAs.
//
// Blocks are persistent: gridDim.x is a multiple of 8 and block b serves the tiles of
// one eighth of the tile sequence (XCD b % 8 under round-robin dispatch, so the
// concurrently resident blocks of an XCD work on neighbouring tiles and share halos
// in that XCD's L2; theta fastest, then phi, then r), stepping by gridDim.x / 8; a block
// whose input is a single slice loads its weights once.
template <int NT, int TJ, int TK, int SIGN, bool AHEAD, class Load, class Finish, class Store>
__device__ __forceinline__ void conv_tiles(const Lv &L, int cin, const bf16 *__restrict__ w, Load load, Finish finish,
                                           Store store)
{
    using T = Tile<TJ, TK>;
    constexpr int PW = T::per_wave;
    extern __shared__ uint4 smem_u4[];
    char *lds = reinterpret_cast<char *>(smem_u4);
    char *ws = lds + T::cells * 32;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int cout = NT * 16;
    const int nslice = cin / 16;
    // 32-bit tile, cell and element indices (the launchers take levels of fewer than 2^31
    // cells); only a cell index times its channel count is formed in 64 bits
    const int ntr = (L.nr + kTR - 1) / kTR, ntj = (L.nt + TJ - 1) / TJ, ntk = (L.np + TK - 1) / TK;
    const int ntiles = ntr * ntj * ntk;
    const int per = gridDim.x >> 3, xcd = blockIdx.x & 7;
    const int t_end = (int)((long)ntiles * (xcd + 1) / 8);
    int tile = (int)((long)ntiles * xcd / 8) + (blockIdx.x >> 3);
    if (tile >= t_end) return;  // uniform over the block
    // tile t -> (tr, tj, tk): theta fastest, then phi, then r
    auto decode = [&](int t, int &r0, int &j0, int &k0) __attribute__((always_inline)) {
        const int q = t / ntj, tr = q / ntk;
        j0 = (t - q * ntj) * TJ;
        k0 = (q - tr * ntk) * TK;
        r0 = tr * kTR;
    };
    constexpr int NL = (T::cells * 2 + kTB - 1) / kTB;   // 16-byte tile loads per thread
    constexpr int NW = (27 * NT * 32 + kTB - 1) / kTB;   // 16-byte weight loads per thread
    // the zero weights of the padding tap 27
    if (tid < NT * 32) *reinterpret_cast<uint4 *>(ws + (27 * NT * 32 + tid) * 16) = make_uint4(0u, 0u, 0u, 0u);
    // per-lane fragment bases: segment q of this wavefront is (rh = q & 1, jj = jw + q / 2, kw)
    const int g0 = wv * PW, jw = (g0 >> 1) % TJ, kw = (g0 >> 1) / TJ;
    const int half = (lane >> 4) & 1;
    const int xbase = (((kw + 1) * T::HJ + (jw + 1)) * T::HR + 1 + (lane & 15)) * 32 + half * 16;
    const int wbase = ((lane >> 5) * NT * 32 + (lane & 31)) * 16;
    float4v acc[PW][NT];
#pragma unroll
    for (int q = 0; q < PW; q++)
#pragma unroll
        for (int t = 0; t < NT; t++) acc[q][t] = float4v{0.f, 0.f, 0.f, 0.f};
    // the global loads of item (tile t, slice sl) into registers, all issued before the
    // LDS stores; load(idx, a, b, c, ch, ok) returns 8 channels of cell (a, b, c), or
    // zeros where !ok (cells outside the grid, which arrive as (0, 0, 0)).  A native
    // vector type with compile-time indices, so the staging stays in registers (the HIP
    // uint4 struct made the compiler keep such arrays in scratch memory).
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    typedef decltype(load(0, 0, 0, 0, 0)) Raw;
    auto fetch = [&](int t, int sl, Raw (&vv)[NL], unsigned &okm) __attribute__((always_inline)) {
        okm = 0u;
        // tile order: theta fastest, then phi, then r, so the blocks resident together
        // share their theta halos and the next wave of blocks finds its phi halo plane in L2
        int r0, j0, k0;
        decode(t, r0, j0, k0);
        static_for<0, NL>([&](auto uc) __attribute__((always_inline)) {
            constexpr int u = decltype(uc)::value;
            const int q = tid + u * kTB;
            const int cell = q >> 1, h = q & 1;
            const int hr = cell % T::HR, hj = (cell / T::HR) % T::HJ, hk = cell / (T::HR * T::HJ);
            int a = r0 + hr - 1, b = j0 + hj - 1, c = k0 + hk - 1;
            c = (c == -1) ? L.np - 1 : (c == L.np ? 0 : c);
            const bool ok = q < T::cells * 2 && (unsigned)a < (unsigned)L.nr && (unsigned)b < (unsigned)L.nt &&
                            (unsigned)c < (unsigned)L.np;
            if (!ok) a = b = c = 0;
            okm |= (unsigned)ok << u;
            vv[u] = load(a + L.nr * (b + L.nt * c), a, b, c, sl * 16 + h * 8);
        });
    };
    auto put = [&](const Raw (&vv)[NL], unsigned okm) __attribute__((always_inline)) {
        static_for<0, NL>([&](auto uc) __attribute__((always_inline)) {
            constexpr int u = decltype(uc)::value;
            const int q = tid + u * kTB;
            if (q < T::cells * 2) *reinterpret_cast<u32x4 *>(lds + q * 16) = finish(vv[u], (okm >> u) & 1u);
        });
    };
    // the weights of slice sl (all 27 taps, fragment order) into registers
    auto fetch_w = [&](int sl, u32x4 (&wr)[NW]) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < NW; u++) {
            const int q = min(tid + u * kTB, 27 * NT * 32 - 1);
            const int l32 = q & 31, tt = (q >> 5) % NT, tap = q / (32 * NT);
            const int co = tt * 16 + (l32 & 15), ci = sl * 16 + (l32 >> 4) * 8;
            wr[u] = *reinterpret_cast<const u32x4 *>(w + ((long)tap * cout + co) * cin + ci);
        }
    };
    auto put_w = [&](const u32x4 (&wr)[NW]) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < NW; u++) {
            const int q = tid + u * kTB;
            if (q < 27 * NT * 32) *reinterpret_cast<u32x4 *>(ws + q * 16) = wr[u];
        }
    };
    // AHEAD (the forward convolutions with 16 output channels: the fine level, where the
    // layer is bound by moving its activations): the next item's tile and weights are
    // loaded into registers before this item's MFMAs, so their latency overlaps the
    // matrix work; otherwise (the wider layers, at the register limit already, and the
    // data gradient, whose loads are converted as they arrive) each item is loaded after
    // the previous one's MFMAs.
    constexpr bool kAhead = AHEAD;
    Raw v[NL];
    u32x4 wr[NW];
    unsigned okm;
    if (kAhead) {
        fetch(tile, 0, v, okm);
        fetch_w(0, wr);
    }
    int s = 0;
    bool first = true;
    for (;;) {
        const int cur = tile;
        const int cs = s;
        if (!kAhead) fetch(cur, cs, v, okm);
        __syncthreads();  // the previous item's MFMAs are done with the LDS tiles
        put(v, okm);
        if (first || nslice > 1) {
            if (!kAhead) fetch_w(cs, wr);
            put_w(wr);
        }
        first = false;
        __syncthreads();
        if (++s == nslice) {
            s = 0;
            tile += per;
        }
        if (kAhead && tile < t_end) {
            fetch(tile, s, v, okm);
            if (nslice > 1) fetch_w(s, wr);
        }
        // Tap pairs p = 0 .. 13, software-pipelined: the LDS fragments of pair p + 1 are
        // requested before the MFMAs of pair p are issued.
        auto frags = [&](auto pc, bf16x8 (&bf)[PW], bf16x8 (&af)[NT]) {
            constexpr int p = decltype(pc)::value;
            constexpr int ta = 2 * p, tb = (2 * p + 1 < 27) ? 2 * p + 1 : 13;
            constexpr int oa = SIGN * (((ta / 9 - 1) * T::HJ + ((ta / 3) % 3 - 1)) * T::HR + (ta % 3 - 1)) * 32;
            constexpr int ob = SIGN * (((tb / 9 - 1) * T::HJ + ((tb / 3) % 3 - 1)) * T::HR + (tb % 3 - 1)) * 32;
            const char *xp = lds + xbase + ((lane < 32) ? oa : ob);
#pragma unroll
            for (int q = 0; q < PW; q++)
                bf[q] = *reinterpret_cast<const bf16x8 *>(xp + ((q >> 1) * T::HR + (q & 1) * 16) * 32);
            const char *wp = ws + wbase + 2 * p * NT * 32 * 16;
#pragma unroll
            for (int t = 0; t < NT; t++) af[t] = *reinterpret_cast<const bf16x8 *>(wp + t * 32 * 16);
        };
        auto mma = [&](const bf16x8 (&bf)[PW], const bf16x8 (&af)[NT]) {
#pragma unroll
            for (int q = 0; q < PW; q++)
#pragma unroll
                for (int t = 0; t < NT; t++)
                    acc[q][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[t], bf[q], acc[q][t], 0, 0, 0);
        };
        bf16x8 b0[PW], a0[NT], b1[PW], a1[NT];
        frags(std::integral_constant<int, 0>{}, b0, a0);
        static_for<0, 7>([&](auto i) {
            constexpr int p = 2 * decltype(i)::value;
            frags(std::integral_constant<int, p + 1>{}, b1, a1);
            __builtin_amdgcn_sched_barrier(0);
            mma(b0, a0);
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (p + 2 < 14) frags(std::integral_constant<int, p + 2>{}, b0, a0);
            __builtin_amdgcn_sched_barrier(0);
            mma(b1, a1);
            __builtin_amdgcn_sched_barrier(0);
        });
        if (cs == nslice - 1) {
            int r0, j0, k0;
            decode(cur, r0, j0, k0);
#pragma unroll
            for (int q = 0; q < PW; q++) {
                const int a = r0 + (q & 1) * 16 + (lane & 15), b = j0 + jw + (q >> 1), c = k0 + kw;
                if (a < L.nr && b < L.nt && c < L.np) {
                    const int idx = a + L.nr * (b + L.nt * c);
#pragma unroll
                    for (int t = 0; t < NT; t++) store(idx, t * 16 + 4 * (lane >> 4), acc[q][t]);
                }
#pragma unroll
                for (int t = 0; t < NT; t++) acc[q][t] = float4v{0.f, 0.f, 0.f, 0.f};
            }
        }
        if (tile >= t_end) break;
    }
}

// ------------------------------------------------- sliding-window convolution
//
// The 16 -> 16 channel layers of the fine level (one input slice) move little data per
// MFMA, and measured on gfx950 the tiled kernel above is bound by the L2 -> L1 requests
// a compute unit can keep in flight (L1 stalled on pending requests 65 % of the time),
// not by HBM or the matrix cores: its 32 x 4 x 4 tiles load 2.4 halo cells per output
// cell.  (Sharing each activation fragment between the three phi offsets, with rolling
// accumulators per output plane, halves the LDS reads but needs more registers than three
// wavefronts per SIMD allow, and measured slower.)  Here a block owns a column of kTR x TJ cells
// (r x theta) over a chunk of kSlideP phi planes and walks it plane by plane, keeping the
// three halo planes a step reads (k - 1, k, k + 1) in a ring in LDS: each step loads one
// new (kTR + 2) x (TJ + 2) plane (1.33 halo cells per output cell with TJ = 8), the one
// the next step needs, into registers before its own MFMAs so the latency overlaps them,
// and the weights stay resident.  The MFMA fragments and their order are those of conv_tiles; only the phi
// offset of a tap becomes the ring slot of its plane.
constexpr int kSlideTJ = 8;   // theta rows of a block
constexpr int kSlideP = 32;   // phi planes of a block

template <int TJ>
struct SlidePlane {
    static constexpr int HR = kTR + 2, HJ = TJ + 2;
    static constexpr int cells = HR * HJ;
    static constexpr int bytes = cells * 32;  // cell-major, 32 bytes (16 bf16 channels) a cell
    static constexpr int per_wave = 2 * TJ / 4;  // 16-cell row segments of a wavefront per plane
    static_assert(TJ % 2 == 0, "a wavefront owns pairs of theta rows");
};

// LDS bytes of one block: the ring of three halo planes plus the weights (28 taps).
template <int TJ>
constexpr size_t slide_lds_bytes() { return 3 * (size_t)SlidePlane<TJ>::bytes + 28 * 512; }

// Forward convolution with 16 input and 16 output channels; load / finish as for
// conv_tiles; store(idx, ch, v, ok, q, k) is called by every lane (ok false for cells
// outside the grid, idx then 0), so an epilogue may exchange values between lanes; q is
// the wavefront's segment (r half q & 1 of theta row 2 wv + q / 2) and k the phi plane,
// in the order the segments and planes are finished.  Item i of the grid: theta tile fastest, then r tile, then phi chunk;
// gridDim.x is a multiple of 8 and the items of one eighth run on one XCD (block b on
// XCD b % 8), so the blocks resident together are neighbours in theta and r and share
// their halos in that XCD's L2.
template <int TJ, class Load, class Finish, class Store>
__device__ __forceinline__ void conv_slide(const Lv &L, const bf16 *__restrict__ w, Load load, Finish finish,
                                           Store store)
{
    using P = SlidePlane<TJ>;
    constexpr int PW = P::per_wave;
    extern __shared__ uint4 smem_u4[];
    char *lds = reinterpret_cast<char *>(smem_u4);
    char *ws = lds + 3 * P::bytes;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int ntr = (L.nr + kTR - 1) / kTR, ntj = (L.nt + TJ - 1) / TJ, nch = (L.np + kSlideP - 1) / kSlideP;
    const int nitems = ntr * ntj * nch;
    const int item = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    if (item >= nitems) return;  // uniform over the block
    const int q0 = item / ntj, tj = item - q0 * ntj, chunk = q0 / ntr, tr = q0 - chunk * ntr;
    const int r0 = tr * kTR, j0 = tj * TJ, k0 = chunk * kSlideP;
    const int k1 = min(L.np, k0 + kSlideP);
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    // weights of all 27 taps in fragment order, and the zero tap 27 that pads the last pair
    constexpr int NW = (27 * 32 + kTB - 1) / kTB;
    if (tid < 32) *reinterpret_cast<u32x4 *>(ws + (27 * 32 + tid) * 16) = u32x4{0u, 0u, 0u, 0u};
#pragma unroll
    for (int u = 0; u < NW; u++) {
        const int q = tid + u * kTB;
        if (q < 27 * 32) {
            const int l32 = q & 31, tap = q >> 5;
            *reinterpret_cast<u32x4 *>(ws + q * 16) =
                *reinterpret_cast<const u32x4 *>(w + (tap * 16 + (l32 & 15)) * 16 + (l32 >> 4) * 8);
        }
    }
    // one halo plane p (phi index, wrapped): loads issued into registers, written to a ring
    // slot later (zeros outside r and theta)
    constexpr int NL = (P::cells * 2 + kTB - 1) / kTB;
    typedef decltype(load(0, 0, 0, 0, 0)) Raw;
    auto fetch = [&](int p, Raw (&vv)[NL], unsigned &okm) __attribute__((always_inline)) {
        okm = 0u;
        const int cp = p < 0 ? p + L.np : (p >= L.np ? p - L.np : p);
        static_for<0, NL>([&](auto uc) __attribute__((always_inline)) {
            constexpr int u = decltype(uc)::value;
            const int q = tid + u * kTB;
            const int cell = q >> 1, h = q & 1;
            const int hr = cell % P::HR, hj = cell / P::HR;
            int a = r0 + hr - 1, b = j0 + hj - 1, c = cp;
            const bool ok = q < P::cells * 2 && (unsigned)a < (unsigned)L.nr && (unsigned)b < (unsigned)L.nt;
            if (!ok) a = b = c = 0;
            okm |= (unsigned)ok << u;
            vv[u] = load(a + L.nr * (b + L.nt * c), a, b, c, h * 8);
        });
    };
    auto put = [&](int slot, const Raw (&vv)[NL], unsigned okm) __attribute__((always_inline)) {
        char *pl = lds + slot * P::bytes;
        static_for<0, NL>([&](auto uc) __attribute__((always_inline)) {
            constexpr int u = decltype(uc)::value;
            const int q = tid + u * kTB;
            if (q < P::cells * 2) *reinterpret_cast<u32x4 *>(pl + q * 16) = finish(vv[u], (okm >> u) & 1u);
        });
    };
    // planes k0 - 1, k0, k0 + 1 in slots 0, 1, 2 (plane p lives in slot (p - k0 + 1) mod 3)
    Raw v[NL];
    unsigned okm;
    fetch(k0 - 1, v, okm);
    put(0, v, okm);
    fetch(k0, v, okm);
    put(1, v, okm);
    fetch(k0 + 1, v, okm);
    put(2, v, okm);
    // fragment bases: segment q of this wavefront is (rh = q & 1, theta row 2 wv + q / 2)
    const int half = (lane >> 4) & 1;
    const int xl = (2 * wv * P::HR + (lane & 15)) * 32 + half * 16;
    const int wbase = ((lane >> 5) * 32 + (lane & 31)) * 16;
    // Step k: the loads of plane k + 2 are issued, the MFMAs of planes k - 1 .. k + 1 run,
    // and after a barrier plane k + 2 replaces plane k - 1 in the ring, before this step's
    // outputs are stored: the wait for its loads then finds nothing younger in flight
    // (loads and stores share one counter, and conditional stores would make it wait for
    // every store of the previous step).
    __syncthreads();
    for (int k = k0; k < k1; k++) {
        const bool more = k + 2 <= k1;
        if (more) fetch(k + 2, v, okm);  // in flight during the MFMAs
        // ring slots of planes k - 1, k, k + 1 (taps with phi offset dk = 0, 1, 2)
        const int sb0 = ((k - k0) % 3) * P::bytes, sb1 = ((k - k0 + 1) % 3) * P::bytes,
                  sb2 = ((k - k0 + 2) % 3) * P::bytes;
        float4v acc[PW];
#pragma unroll
        for (int q = 0; q < PW; q++) acc[q] = float4v{0.f, 0.f, 0.f, 0.f};
        auto frags = [&](auto pc, bf16x8 (&bf)[PW], bf16x8 &af) {
            constexpr int p = decltype(pc)::value;
            constexpr int ta = 2 * p, tb = (2 * p + 1 < 27) ? 2 * p + 1 : 13;
            constexpr int oa = (((ta / 3) % 3) * P::HR + ta % 3) * 32;
            constexpr int ob = (((tb / 3) % 3) * P::HR + tb % 3) * 32;
            const int sa = ta / 9 == 0 ? sb0 : (ta / 9 == 1 ? sb1 : sb2);
            const int sbb = tb / 9 == 0 ? sb0 : (tb / 9 == 1 ? sb1 : sb2);
            const char *xp = lds + xl + ((lane < 32) ? sa + oa : sbb + ob);
#pragma unroll
            for (int q = 0; q < PW; q++)
                bf[q] = *reinterpret_cast<const bf16x8 *>(xp + ((q >> 1) * P::HR + (q & 1) * 16) * 32);
            af = *reinterpret_cast<const bf16x8 *>(ws + wbase + 2 * p * 32 * 16);
        };
        auto mma = [&](const bf16x8 (&bf)[PW], const bf16x8 &af) {
#pragma unroll
            for (int q = 0; q < PW; q++) acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf[q], acc[q], 0, 0, 0);
        };
        bf16x8 b0[PW], b1[PW], a0, a1;
        frags(std::integral_constant<int, 0>{}, b0, a0);
        static_for<0, 7>([&](auto i) {
            constexpr int p = 2 * decltype(i)::value;
            frags(std::integral_constant<int, p + 1>{}, b1, a1);
            __builtin_amdgcn_sched_barrier(0);
            mma(b0, a0);
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (p + 2 < 14) frags(std::integral_constant<int, p + 2>{}, b0, a0);
            __builtin_amdgcn_sched_barrier(0);
            mma(b1, a1);
            __builtin_amdgcn_sched_barrier(0);
        });
        __syncthreads();  // every wavefront is done with the slot of plane k - 1
        if (more) put((k - k0) % 3, v, okm);
#pragma unroll
        for (int q = 0; q < PW; q++) {
            const int a = r0 + (q & 1) * 16 + (lane & 15), b = j0 + 2 * wv + (q >> 1);
            const bool ok = a < L.nr && b < L.nt;
            store(ok ? a + L.nr * (b + L.nt * k) : 0, 4 * (lane >> 4), acc[q], ok, q, k);
        }
        __syncthreads();  // plane k + 2 is in the ring for the next step
    }
}

// y = act(conv([up?(x1), x2], w) + bias) with NT * 16 output channels.  x1 has c1
// channels and lives on the level of y (up1 = 0) or on the next coarser level
// (up1 = 1, read through nearest-neighbour upsampling); x2 (c2 channels, may be 0) on
// the level of y.  Writes bf16 y and/or fp32 yf.
template <int NT, int TJ, int TK, bool SLIDE = false>
__global__ __launch_bounds__(kTB) __attribute__((amdgpu_waves_per_eu(NT == 1 ? 3 : 2, 8))) void k_conv_fwd(
    Lv L, const bf16 *__restrict__ x1, int c1, int up1, const bf16 *__restrict__ x2, int c2,
    const bf16 *__restrict__ w, const float *__restrict__ bias, int relu, bf16 *__restrict__ y, float *__restrict__ yf)
{
    const int cr = L.nr >> 1, ct = L.nt >> 1;
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    auto load = [&](int idx, int a, int b, int c, int ch) -> u32x4 {
        const bf16 *p;
        if (ch < c1) {
            const int e = up1 ? (a >> 1) + cr * ((b >> 1) + ct * (c >> 1)) : idx;
            p = x1 + (size_t)e * c1 + ch;
        } else {
            p = x2 + (size_t)idx * c2 + (ch - c1);
        }
        return *reinterpret_cast<const u32x4 *>(p);
    };
    auto finish = [](const u32x4 &x, bool ok) -> u32x4 { return ok ? x : u32x4{0u, 0u, 0u, 0u}; };
    const int cout = NT * 16;
    // the bias of this lane's output channels t 16 + 4 (lane / 16) .. + 3 of each output
    // tile t, loaded once (the epilogue then waits for no memory)
    float4 bsel[NT];
#pragma unroll
    for (int t = 0; t < NT; t++)
        bsel[t] = bias ? *reinterpret_cast<const float4 *>(bias + t * 16 + 4 * ((threadIdx.x & 63) >> 4))
                       : make_float4(0.f, 0.f, 0.f, 0.f);
    auto store = [&](int idx, int co, const float4v &v) {
        const float4 bb = bsel[co >> 4];
        float o[4] = {v[0] + bb.x, v[1] + bb.y, v[2] + bb.z, v[3] + bb.w};
        if (relu) {  // a select, no branch; NaN passes (the comparison is false)
#pragma unroll
            for (int i = 0; i < 4; i++) o[i] = o[i] < 0.0f ? 0.0f : o[i];
        }
        if (y) *reinterpret_cast<uint2 *>(y + (size_t)idx * cout + co) = make_uint2(pack_bf16(o[0], o[1]), pack_bf16(o[2], o[3]));
        if (yf) *reinterpret_cast<float4 *>(yf + (size_t)idx * cout + co) = make_float4(o[0], o[1], o[2], o[3]);
    };
    if constexpr (SLIDE)  // NT = 1, c1 + c2 = 16
        conv_slide<TJ>(L, w, load, finish, [&](int idx, int co, const float4v &v, bool ok, int, int) {
            if (ok) store(idx, co, v);
        });
    else conv_tiles<NT, TJ, TK, 1, false>(L, c1 + c2, w, load, finish, store);
}

// Layer 0 of the preconditioner's application with its input built on the fly: channel
// 0 is the residual r (fp32) times scale[0] (to unit RMS) rounded to bf16, channels 1..7
// come from X (the operator features of k_features and zeros; X's own channel 0 is not
// read), channels 8..15 are zero and not loaded.  The same operands, bit for bit, as
// k_set_input followed by k_conv_fwd<1,4,4> on X, without writing X (16 output
// channels, bias, ReLU, bf16 out).
template <bool SLIDE>
__global__ __launch_bounds__(kTB) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_conv_fwd_in(
    Lv L, const bf16 *__restrict__ X, const float *__restrict__ r, const double *__restrict__ scale,
    const bf16 *__restrict__ w, const float *__restrict__ bias, bf16 *__restrict__ y)
{
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    const double sc = scale[0];
    // both halves of a cell read its channels 0..7 (the same 16 bytes, so no extra
    // traffic); the upper half is then zeroed when the tile is written
    struct Raw {
        u32x4 x;
        float r;
        int lower;
    };
    auto load = [&](int idx, int, int, int, int ch) -> Raw {
        return Raw{*reinterpret_cast<const u32x4 *>(X + (size_t)idx * 16), r[idx], ch == 0};
    };
    auto finish = [&](const Raw &v, bool ok) -> u32x4 {
        u32x4 x = v.x;
        x[0] = (x[0] & 0xFFFF0000u) | f2bf((float)((double)v.r * sc));
        return ok && v.lower ? x : u32x4{0u, 0u, 0u, 0u};
    };
    const float4 bb = *reinterpret_cast<const float4 *>(bias + 4 * ((threadIdx.x & 63) >> 4));
    auto store = [&](int idx, int co, const float4v &v) {
        float o[4] = {v[0] + bb.x, v[1] + bb.y, v[2] + bb.z, v[3] + bb.w};
#pragma unroll
        for (int i = 0; i < 4; i++) o[i] = o[i] < 0.0f ? 0.0f : o[i];
        *reinterpret_cast<uint2 *>(y + (size_t)idx * 16 + co) = make_uint2(pack_bf16(o[0], o[1]), pack_bf16(o[2], o[3]));
    };
    if constexpr (SLIDE)
        conv_slide<kSlideTJ>(L, w, load, finish, [&](int idx, int co, const float4v &v, bool ok, int, int) {
            if (ok) store(idx, co, v);
        });
    else conv_tiles<1, 4, 4, 1, false>(L, 16, w, load, finish, store);
}

// The network's last two layers in one pass, for the forward passes whose activations
// are not kept for a backward pass: h = relu(conv(x, w) + bias) (16 -> 16, the sliding
// kernel) rounded to bf16, then z = wo . h + bo (the 1x1 output layer, fp32) instead of
// writing h.  The same operands and the same fp32 operations in the same order as
// k_conv_fwd followed by k_out_fwd, so z is bit for bit theirs.  Each lane ends with 4
// channels of one cell; the cell's 16 channels are gathered into lanes 0..15 by
// ds_bpermute, which every lane executes.
__global__ __launch_bounds__(kTB) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_conv_fwd_head(
    Lv L, const bf16 *__restrict__ x, const bf16 *__restrict__ w, const float *__restrict__ bias,
    const bf16 *__restrict__ wo, const float *__restrict__ bo, const double *__restrict__ scale, float *__restrict__ z)
{
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    auto load = [&](int idx, int, int, int, int ch) -> u32x4 {
        return *reinterpret_cast<const u32x4 *>(x + (size_t)idx * 16 + ch);
    };
    auto finish = [](const u32x4 &v, bool ok) -> u32x4 { return ok ? v : u32x4{0u, 0u, 0u, 0u}; };
    const int lane = threadIdx.x & 63, e = lane & 15;
    const float4 bb = *reinterpret_cast<const float4 *>(bias + 4 * (lane >> 4));
    float wof[16];
#pragma unroll
    for (int q = 0; q < 16; q++) wof[q] = bf2f(wo[q]);
    const float b0 = bo[0];
    const double sc = scale ? scale[1] : 1.0;
    auto store = [&](int idx, int, const float4v &v, bool ok, int, int) {
        float o[4] = {v[0] + bb.x, v[1] + bb.y, v[2] + bb.z, v[3] + bb.w};
#pragma unroll
        for (int i = 0; i < 4; i++) o[i] = o[i] < 0.0f ? 0.0f : o[i];
        const unsigned d0 = pack_bf16(o[0], o[1]), d1 = pack_bf16(o[2], o[3]);
        unsigned hv[8];
        hv[0] = d0;
        hv[1] = d1;
#pragma unroll
        for (int g = 1; g < 4; g++) {
            hv[2 * g] = (unsigned)__builtin_amdgcn_ds_bpermute((e + 16 * g) * 4, (int)d0);
            hv[2 * g + 1] = (unsigned)__builtin_amdgcn_ds_bpermute((e + 16 * g) * 4, (int)d1);
        }
        if (lane < 16 && ok) {
            float s = b0;
#pragma unroll
            for (int q = 0; q < 16; q++)
                s = fmaf(wof[q], bf2f((bf16)(q & 1 ? hv[q >> 1] >> 16 : hv[q >> 1] & 0xFFFFu)), s);
            z[idx] = scale ? (float)((double)s * sc) : s;
        }
    };
    conv_slide<kSlideTJ>(L, w, load, finish, store);
}

// y = relu(conv(x, w) + bias) (16 -> 16, the sliding kernel, bf16 out) and its 2x2x2
// average pool yp on the next coarser level in the same pass (the fine level's second
// layer, whose output is both the skip connection and the input of level 1).  The block
// walks phi planes in pairs from an even plane, each wavefront owns a pair of theta rows
// (an even one first) and the two cells of an r pair sit in lanes l and l ^ 1, so the
// eight children of a coarse cell meet in the even lane as r, theta, phi advance: the
// same bf16 values summed in fp32 in the same order as k_pool, hence the same bits.  Every
// dimension of the level is even.
__global__ __launch_bounds__(kTB) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_conv_fwd_pool(
    Lv L, const bf16 *__restrict__ x, const bf16 *__restrict__ w, const float *__restrict__ bias,
    bf16 *__restrict__ y, bf16 *__restrict__ yp)
{
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    auto load = [&](int idx, int, int, int, int ch) -> u32x4 {
        return *reinterpret_cast<const u32x4 *>(x + (size_t)idx * 16 + ch);
    };
    auto finish = [](const u32x4 &v, bool ok) -> u32x4 { return ok ? v : u32x4{0u, 0u, 0u, 0u}; };
    const int lane = threadIdx.x & 63;
    const float4 bb = *reinterpret_cast<const float4 *>(bias + 4 * (lane >> 4));
    const int cr = L.nr >> 1, ct = L.nt >> 1;
    float ps[2][4];  // the running sums of this lane's 4 channels, per r half of the segments
    auto store = [&](int idx, int co, const float4v &v, bool ok, int q, int k) {
        float o[4] = {v[0] + bb.x, v[1] + bb.y, v[2] + bb.z, v[3] + bb.w};
#pragma unroll
        for (int i = 0; i < 4; i++) o[i] = o[i] < 0.0f ? 0.0f : o[i];
        const unsigned d0 = pack_bf16(o[0], o[1]), d1 = pack_bf16(o[2], o[3]);
        if (ok) *reinterpret_cast<uint2 *>(y + (size_t)idx * 16 + co) = make_uint2(d0, d1);
        const float h[4] = {bf2f((bf16)(d0 & 0xFFFFu)), bf2f((bf16)(d0 >> 16)), bf2f((bf16)(d1 & 0xFFFFu)),
                            bf2f((bf16)(d1 >> 16))};
        const int rh = q & 1;
        if (q < 2 && (k & 1) == 0) {
#pragma unroll
            for (int i = 0; i < 4; i++) ps[rh][i] = 0.0f;
        }
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const float nb = __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(h[i]), 0x041F));  // lane ^ 1
            ps[rh][i] += h[i];
            ps[rh][i] += nb;
        }
        if (q >= 2 && (k & 1) == 1 && (lane & 1) == 0 && ok) {
            const int b = (idx / L.nr) % L.nt, a = idx % L.nr;
            const size_t g = (size_t)((a >> 1) + cr * ((b >> 1) + ct * (k >> 1)));
            *reinterpret_cast<uint2 *>(yp + g * 16 + co) =
                make_uint2((unsigned)f2bf(ps[rh][0] * 0.125f) | ((unsigned)f2bf(ps[rh][1] * 0.125f) << 16),
                           (unsigned)f2bf(ps[rh][2] * 0.125f) | ((unsigned)f2bf(ps[rh][3] * 0.125f) << 16));
        }
    };
    conv_slide<kSlideTJ>(L, w, load, finish, store);
}

// ------------------------------------------ sliding decoder convolution (fine level)
//
// The fine level's decoder layer: y = relu(conv([up(x1), x2], w) + bias) with x1 the 32
// channels of level 1 read through nearest-neighbour upsampling, x2 the 16 skip channels
// and 16 output channels.  A block of kDecWaves wavefronts owns a column of kTR x
// kDecTJ cells (r x theta) over a chunk of kSlideP phi planes and walks it plane by
// plane like conv_slide.  The skip channels keep conv_slide's ring of three fine halo
// planes.  The upsampled channels are never expanded: the ring holds the coarse planes
// themselves (a (kTR/2 + 2) x (kDecTJ/2 + 2) halo plane covers the fine (kTR + 2) x (kDecTJ + 2)
// plane), one new coarse plane every second step (two slots: a fine step reads two coarse
// planes, and the new one replaces the older after the step's MFMAs), and each fine
// cell's tap reads its coarse parent.  For those channels K = 32 is one tap x the 32 channels (lanes 0..31
// the first 16, lanes 32..63 the other 16), so 27 MFMAs per segment and no padding tap;
// the skip channels use conv_slide's tap pairs.  Same operands and the same FP32 sums as
// the tiled kernel, only ordered differently.
constexpr int kDecWaves = 12;
constexpr int kDecTB = 64 * kDecWaves;
constexpr int kDecTJ = 2 * kDecWaves;  // theta rows of a block (two per wavefront)

struct DecGeom {
    static constexpr int HR = kTR + 2, HJ = kDecTJ + 2;     // fine halo plane
    static constexpr int fine_bytes = HR * HJ * 32;         // 16 channels a cell
    static constexpr int CR = kTR / 2 + 2, CJ = kDecTJ / 2 + 2;  // coarse halo plane
    static constexpr int cslice_bytes = CR * CJ * 32;       // one 16-channel slice
    static constexpr int coarse_bytes = 2 * cslice_bytes;
    static constexpr int wskip_bytes = 28 * 32 * 16;        // tap pairs, zero tap 27
    static constexpr int wup_bytes = 27 * 64 * 16;
    static constexpr int lds = 3 * fine_bytes + 2 * coarse_bytes + wskip_bytes + wup_bytes;
};

__global__ __launch_bounds__(kDecTB) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_conv_fwd_dec(
    Lv L, const bf16 *__restrict__ x1, const bf16 *__restrict__ x2, const bf16 *__restrict__ w,
    const float *__restrict__ bias, int relu, bf16 *__restrict__ y, float *__restrict__ yf)
{
    using G = DecGeom;
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    extern __shared__ uint4 smem_u4[];
    char *lds = reinterpret_cast<char *>(smem_u4);
    char *cring = lds + 3 * G::fine_bytes;
    char *wsk = cring + 2 * G::coarse_bytes;
    char *wup = wsk + G::wskip_bytes;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int cr = L.nr >> 1, ct = L.nt >> 1, cp = L.np >> 1;
    const int ntr = (L.nr + kTR - 1) / kTR, ntj = (L.nt + kDecTJ - 1) / kDecTJ, nch = (L.np + kSlideP - 1) / kSlideP;
    const int nitems = ntr * ntj * nch;
    const int item = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    if (item >= nitems) return;  // uniform over the block
    const int q0 = item / ntj, tj = item - q0 * ntj, chunk = q0 / ntr, tr = q0 - chunk * ntr;
    const int r0 = tr * kTR, j0 = tj * kDecTJ, k0 = chunk * kSlideP;  // all even
    const int k1 = min(L.np, k0 + kSlideP);
    const int c0 = (k0 >> 1) - 1;  // coarse plane c lives in ring slot (c - c0) mod 2
    // weights: skip channels 32..47 as tap pairs [tap][co + 16 half], up channels 0..31 as
    // [tap][co + 16 (ci / 8)]
    if (tid < 32) *reinterpret_cast<u32x4 *>(wsk + (27 * 32 + tid) * 16) = u32x4{0u, 0u, 0u, 0u};
    for (int q = tid; q < 27 * 32 + 27 * 64; q += kDecTB) {
        if (q < 27 * 32) {
            const int l32 = q & 31, tap = q >> 5;
            *reinterpret_cast<u32x4 *>(wsk + q * 16) =
                *reinterpret_cast<const u32x4 *>(w + (tap * 16 + (l32 & 15)) * 48 + 32 + (l32 >> 4) * 8);
        } else {
            const int u = q - 27 * 32, l64 = u & 63, tap = u >> 6;
            *reinterpret_cast<u32x4 *>(wup + u * 16) =
                *reinterpret_cast<const u32x4 *>(w + (tap * 16 + (l64 & 15)) * 48 + (l64 >> 4) * 8);
        }
    }
    // fine skip plane p (wrapped in phi): 16-byte loads into registers, zeros outside r, theta
    constexpr int NL = (G::HR * G::HJ * 2 + kDecTB - 1) / kDecTB;
    auto fetch = [&](int p, u32x4 (&vv)[NL], unsigned &okm) __attribute__((always_inline)) {
        okm = 0u;
        const int pp = p < 0 ? p + L.np : (p >= L.np ? p - L.np : p);
        static_for<0, NL>([&](auto uc) __attribute__((always_inline)) {
            constexpr int u = decltype(uc)::value;
            const int q = tid + u * kDecTB;
            const int cell = q >> 1, h = q & 1;
            const int hr = cell % G::HR, hj = cell / G::HR;
            int a = r0 + hr - 1, b = j0 + hj - 1;
            const bool ok = q < G::HR * G::HJ * 2 && (unsigned)a < (unsigned)L.nr && (unsigned)b < (unsigned)L.nt;
            const int idx = ok ? a + L.nr * (b + L.nt * pp) : 0;
            okm |= (unsigned)ok << u;
            vv[u] = *reinterpret_cast<const u32x4 *>(x2 + (size_t)idx * 16 + h * 8);
        });
    };
    auto put = [&](int slot, const u32x4 (&vv)[NL], unsigned okm) __attribute__((always_inline)) {
        char *pl = lds + slot * G::fine_bytes;
        static_for<0, NL>([&](auto uc) __attribute__((always_inline)) {
            constexpr int u = decltype(uc)::value;
            const int q = tid + u * kDecTB;
            const int cell = q >> 1, hr = cell % G::HR, hj = cell / G::HR;
            const int pos = (hr & 1) ? G::HR / 2 + (hr >> 1) : (hr >> 1);  // even cells first
            if (q < G::HR * G::HJ * 2)
                *reinterpret_cast<u32x4 *>(pl + ((hj * G::HR + pos) * 2 + (q & 1)) * 16) =
                    ((okm >> u) & 1u) ? vv[u] : u32x4{0u, 0u, 0u, 0u};
        });
    };
    // coarse plane c (wrapped): 18 x 10 cells x 64 bytes, four 16-byte pieces a cell
    // (slice s = piece / 2, half h = piece % 2) stored slice-major, 32 bytes a cell
    constexpr int NC = (G::CR * G::CJ * 4 + kDecTB - 1) / kDecTB;
    auto fetch_c = [&](int c, u32x4 (&vv)[NC], unsigned &okm) __attribute__((always_inline)) {
        okm = 0u;
        const int cc = c < 0 ? c + cp : (c >= cp ? c - cp : c);
        static_for<0, NC>([&](auto uc) __attribute__((always_inline)) {
            constexpr int u = decltype(uc)::value;
            const int q = tid + u * kDecTB;
            const int cell = q >> 2, piece = q & 3;
            const int hr = cell % G::CR, hj = cell / G::CR;
            const int a = (r0 >> 1) - 1 + hr, b = (j0 >> 1) - 1 + hj;
            const bool ok = q < G::CR * G::CJ * 4 && (unsigned)a < (unsigned)cr && (unsigned)b < (unsigned)ct;
            const int idx = ok ? a + cr * (b + ct * cc) : 0;
            okm |= (unsigned)ok << u;
            vv[u] = *reinterpret_cast<const u32x4 *>(x1 + (size_t)idx * 32 + piece * 8);
        });
    };
    auto put_c = [&](int slot, const u32x4 (&vv)[NC], unsigned okm) __attribute__((always_inline)) {
        char *pl = cring + slot * G::coarse_bytes;
        static_for<0, NC>([&](auto uc) __attribute__((always_inline)) {
            constexpr int u = decltype(uc)::value;
            const int q = tid + u * kDecTB;
            const int cell = q >> 2, piece = q & 3;
            if (q < G::CR * G::CJ * 4)
                *reinterpret_cast<u32x4 *>(pl + (piece >> 1) * G::cslice_bytes + cell * 32 + (piece & 1) * 16) =
                    ((okm >> u) & 1u) ? vv[u] : u32x4{0u, 0u, 0u, 0u};
        });
    };
    // prologue: fine planes k0 - 1 .. k0 + 1 in slots 0..2, coarse planes c0, c0 + 1
    {
        u32x4 v[NL];
        unsigned okm;
        fetch(k0 - 1, v, okm);
        put(0, v, okm);
        fetch(k0, v, okm);
        put(1, v, okm);
        fetch(k0 + 1, v, okm);
        put(2, v, okm);
        u32x4 vc[NC];
        fetch_c(c0, vc, okm);
        put_c(0, vc, okm);
        fetch_c(c0 + 1, vc, okm);
        put_c(1, vc, okm);
    }
    const float4 bb = bias ? *reinterpret_cast<const float4 *>(bias + 4 * (lane >> 4)) : make_float4(0.f, 0.f, 0.f, 0.f);
    // Fragment bases.  Segment q of this wavefront is the cells of parity s = q & 1 of the
    // 32-cell radial row of theta row 2 wv + q / 2: lane l holds cell 2 (l % 16) + s.  So
    // the 16 lanes of a fragment read 16 distinct coarse parents for every di (with lane =
    // cell, pairs of lanes would read the same parent, which the LDS serves as a conflict),
    // and in the fine ring, whose rows hold the even halo cells before the odd ones, 16
    // consecutive cells: the offset of a tap is k + C(s, di) with k = l % 16, compile-time.
    constexpr int PW = 4;
    const int k16 = lane & 15;
    const int xl = (2 * wv * G::HR + k16) * 32 + ((lane >> 4) & 1) * 16;
    const int wbs = ((lane >> 5) * 32 + (lane & 31)) * 16;
    const int cl = (lane >> 5) * G::cslice_bytes + ((lane >> 4) & 1) * 16 + ((wv + 1) * G::CR + k16 + 1) * 32;
    u32x4 v[NL], vc[NC];
    unsigned okm = 0u, okc = 0u;
    __syncthreads();
    for (int k = k0; k < k1; k++) {
        const bool more = k + 2 <= k1;
        const bool cmore = ((k & 1) == 0) && k + 1 < k1;
        if (more) fetch(k + 2, v, okm);            // in flight during the MFMAs
        if (cmore) fetch_c((k >> 1) + 1, vc, okc);
        const int sb0 = ((k - k0) % 3) * G::fine_bytes, sb1 = ((k - k0 + 1) % 3) * G::fine_bytes,
                  sb2 = ((k - k0 + 2) % 3) * G::fine_bytes;
        // coarse ring slots of the planes under fine planes k - 1, k, k + 1
        const int cs0 = ((((k - 1) >> 1) - c0) & 1) * G::coarse_bytes, cs1 = (((k >> 1) - c0) & 1) * G::coarse_bytes,
                  cs2 = ((((k + 1) >> 1) - c0) & 1) * G::coarse_bytes;
        float4v acc[PW];
#pragma unroll
        for (int q = 0; q < PW; q++) acc[q] = float4v{0.f, 0.f, 0.f, 0.f};
        // halo position of the fine neighbour of cell 2 k + s through di, minus k
        auto cpos = [](int s, int di) constexpr { return s == 0 ? (di == 0 ? G::HR / 2 : (di > 0 ? 1 : 0))
                                                                 : (di == 0 ? 1 : G::HR / 2 + (di > 0 ? 1 : 0)); };
        // group g < 27: up tap g; g >= 27: skip tap pair g - 27
        auto frags = [&](auto gc, bf16x8 (&bf)[PW], bf16x8 &af) __attribute__((always_inline)) {
            constexpr int g = decltype(gc)::value;
            if constexpr (g < 27) {
                constexpr int di = g % 3 - 1, dj = (g / 3) % 3 - 1, dk = g / 9;
                const char *xp = cring + (dk == 0 ? cs0 : (dk == 1 ? cs1 : cs2)) + cl;
                static_for<0, PW>([&](auto qc) __attribute__((always_inline)) {
                    constexpr int q = decltype(qc)::value, sp = q & 1;
                    // the coarse parent of fine cell 2 k + sp + di is k + (sp + di) >> 1
                    constexpr int off = ((((q >> 1) + dj) >> 1) * G::CR + ((sp + di) >> 1)) * 32;
                    bf[q] = *reinterpret_cast<const bf16x8 *>(xp + off);
                });
                af = *reinterpret_cast<const bf16x8 *>(wup + (g * 64 + lane) * 16);
            } else {
                constexpr int p = g - 27;
                constexpr int ta = 2 * p, tb = (2 * p + 1 < 27) ? 2 * p + 1 : 13;
                constexpr int dia = ta % 3 - 1, dib = tb % 3 - 1;
                constexpr int ra = ((ta / 3) % 3) * G::HR * 32, rb = ((tb / 3) % 3) * G::HR * 32;
                const int sa = (ta / 9 == 0 ? sb0 : (ta / 9 == 1 ? sb1 : sb2)) + ra;
                const int sbb = (tb / 9 == 0 ? sb0 : (tb / 9 == 1 ? sb1 : sb2)) + rb;
                // the two parities' bases (the tap pair's halves differ in di)
                const char *x0 = lds + xl + ((lane < 32) ? sa + cpos(0, dia) * 32 : sbb + cpos(0, dib) * 32);
                const char *x1 = lds + xl + ((lane < 32) ? sa + cpos(1, dia) * 32 : sbb + cpos(1, dib) * 32);
                static_for<0, PW>([&](auto qc) __attribute__((always_inline)) {
                    constexpr int q = decltype(qc)::value;
                    bf[q] = *reinterpret_cast<const bf16x8 *>(((q & 1) ? x1 : x0) + (q >> 1) * G::HR * 32);
                });
                af = *reinterpret_cast<const bf16x8 *>(wsk + wbs + 2 * p * 32 * 16);
            }
        };
        auto mma = [&](const bf16x8 (&bf)[PW], const bf16x8 &af) __attribute__((always_inline)) {
#pragma unroll
            for (int q = 0; q < PW; q++) acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf[q], acc[q], 0, 0, 0);
        };
        constexpr int NG = 27 + 14;
        bf16x8 bA[PW], bB[PW], aA, aB;
        frags(std::integral_constant<int, 0>{}, bA, aA);
        static_for<0, NG>([&](auto gc) __attribute__((always_inline)) {
            constexpr int g = decltype(gc)::value;
            if constexpr (g % 2 == 0) {
                if constexpr (g + 1 < NG) frags(std::integral_constant<int, g + 1>{}, bB, aB);
                __builtin_amdgcn_sched_barrier(0);
                mma(bA, aA);
                __builtin_amdgcn_sched_barrier(0);
            } else {
                if constexpr (g + 1 < NG) frags(std::integral_constant<int, g + 1>{}, bA, aA);
                __builtin_amdgcn_sched_barrier(0);
                mma(bB, aB);
                __builtin_amdgcn_sched_barrier(0);
            }
        });
        __syncthreads();  // every wavefront is done with the slots being replaced
        if (more) put((k - k0) % 3, v, okm);
        if (cmore) put_c(((k >> 1) + 1 - c0) & 1, vc, okc);
#pragma unroll
        for (int q = 0; q < PW; q++) {
            const int a = r0 + 2 * k16 + (q & 1), b = j0 + 2 * wv + (q >> 1);
            if (a < L.nr && b < L.nt) {
                const size_t idx = (size_t)(a + L.nr * (b + L.nt * k));
                const int co = 4 * (lane >> 4);
                float o[4] = {acc[q][0] + bb.x, acc[q][1] + bb.y, acc[q][2] + bb.z, acc[q][3] + bb.w};
                if (relu) {
#pragma unroll
                    for (int i = 0; i < 4; i++) o[i] = o[i] < 0.0f ? 0.0f : o[i];
                }
                if (y) *reinterpret_cast<uint2 *>(y + idx * 16 + co) = make_uint2(pack_bf16(o[0], o[1]), pack_bf16(o[2], o[3]));
                if (yf) *reinterpret_cast<float4 *>(yf + idx * 16 + co) = make_float4(o[0], o[1], o[2], o[3]);
            }
        }
        __syncthreads();  // the new planes are in the rings for the next step
    }
}

// ------------------------------------------------------------ data gradient

// dX = conv^T(dYm, w) for the concatenated input [up?(x1), x2] of a convolution with
// cout output channels (dYm = dY masked by the layer's ReLU output y when y != 0).
// Output at the level of dY, NT * 16 input channels: channels < c1 to d1 ([n][c1];
// for an upsampled x1 this is the gradient of the upsampled tensor, folded onto the
// coarse level by k_up_bwd), the rest to d2 ([n][c2]).  Uses the transposed weights
// wt[tap][ci][co], i.e. the forward layout with the roles of ci and co exchanged.
template <int NT, int TJ, int TK>
__global__ __launch_bounds__(kTB) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_conv_bwd_data(
    Lv L, const float *__restrict__ dy, const bf16 *__restrict__ yout, int cout, const bf16 *__restrict__ wt, int c1,
    float *__restrict__ d1, int c2, float *__restrict__ d2)
{
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    auto load = [&](int idx, int, int, int, int ch) -> u32x4 {
        const float4 g0 = *reinterpret_cast<const float4 *>(dy + (size_t)idx * cout + ch);
        const float4 g1 = *reinterpret_cast<const float4 *>(dy + (size_t)idx * cout + ch + 4);
        float f[8] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w};
        if (yout) {
            const uint4 u = *reinterpret_cast<const uint4 *>(yout + (size_t)idx * cout + ch);
            const bf16 *h = reinterpret_cast<const bf16 *>(&u);
#pragma unroll
            for (int q = 0; q < 8; q++)
                if (!(bf2f(h[q]) > 0.0f)) f[q] = 0.0f;
        }
        return u32x4{pack_bf16(f[0], f[1]), pack_bf16(f[2], f[3]), pack_bf16(f[4], f[5]), pack_bf16(f[6], f[7])};
    };
    auto finish = [](const u32x4 &x, bool ok) -> u32x4 { return ok ? x : u32x4{0u, 0u, 0u, 0u}; };
    auto store = [&](int idx, int ci, const float4v &v) {
        const float4 o = make_float4(v[0], v[1], v[2], v[3]);
        if (ci < c1) *reinterpret_cast<float4 *>(d1 + (size_t)idx * c1 + ci) = o;
        else *reinterpret_cast<float4 *>(d2 + (size_t)idx * c2 + (ci - c1)) = o;
    };
    conv_tiles<NT, TJ, TK, -1, false>(L, cout, wt, load, finish, store);
}

// -------------------------------------------------------- weight gradient

// dW[tap][co][ci] = sum over cells of dYm[cell][co] x[nb(cell, tap)][ci], tiled: a block
// owns a 16-channel input slice (blockIdx.y) and walks tiles of kTR x 2 x 2 output
// cells (4 radial rows of 32 cells), blockIdx.x, blockIdx.x + gridDim.x, ...  Per tile
// it stages in LDS the masked output gradient transposed, dyT[co][cell], and three
// r-shifted transposed copies of the input slice, xsT[di][phi row][theta row][ci][i]
// (zero outside r and theta, wrapped in phi), so every MFMA operand is an aligned
// 16-byte read: v_mfma_f32_16x16x32_bf16 with M = co, N = ci, K = the 32 cells of one
// radial row; A[co][cells] from dyT, B[cells][ci] from the copy of the tap's radial
// shift at the tap's theta/phi row.  Wavefront w accumulates taps w, w + 4, ...; the
// block's partial sums go to part[blockIdx.x][tap][co][ci] (summed in a fixed order
// afterwards, so the result is deterministic).
constexpr int kWRowCells = 4 * kTR;          // cells of a tile (2 x 2 rows)
constexpr int kWLdy = kWRowCells + 8;        // dyT row length (bf16), padded against bank conflicts
constexpr int kWLx = kTR + 8;                // xsT row length (bf16), padded
constexpr int kWXRows = 3 * 4 * 4 * 16;      // (di, hk, hj, ci) rows of xsT

template <int NTO>
constexpr size_t wgrad_lds_bytes() { return ((size_t)NTO * 16 * kWLdy + (size_t)kWXRows * kWLx) * 2; }

template <int NTO>
__global__ __launch_bounds__(kTB) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_conv_wgrad(
    Lv L, const float *__restrict__ dy, const bf16 *__restrict__ yout, const bf16 *__restrict__ x1, int c1,
    int up1, const bf16 *__restrict__ x2, int c2, float *__restrict__ part)
{
    extern __shared__ uint4 smem_u4[];
    bf16 *dyT = reinterpret_cast<bf16 *>(smem_u4);
    bf16 *xsT = dyT + NTO * 16 * kWLdy;
    constexpr int cout = NTO * 16;
    const int cin = c1 + c2, sl = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int cr = L.nr >> 1, ct = L.nt >> 1;
    const int ntr = (L.nr + kTR - 1) / kTR, ntj = (L.nt + 1) / 2, ntk = (L.np + 1) / 2;
    const long ntiles = (long)ntr * ntj * ntk;
    float4v acc[7][NTO];
#pragma unroll
    for (int q = 0; q < 7; q++)
#pragma unroll
        for (int t = 0; t < NTO; t++) acc[q][t] = float4v{0.f, 0.f, 0.f, 0.f};
    for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int tj = (int)(tile % ntj), tk = (int)((tile / ntj) % ntk), tr = (int)(tile / ((long)ntj * ntk));
        const int r0 = tr * kTR, j0 = tj * 2, k0 = tk * 2;
        __syncthreads();  // the previous tile's MFMAs are done with LDS
        // dyT[co][row * 32 + i] = dY[cell][co] masked by y > 0 (bf16); i fastest over lanes
        for (int it = tid; it < kWRowCells * (cout / 8); it += kTB) {
            const int i = it % kTR, row = (it / kTR) % 4, cg = it / kWRowCells;
            const int a = r0 + i, b = j0 + (row & 1), c = k0 + (row >> 1);
            float f[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (a < L.nr && b < L.nt && c < L.np) {
                const long idx = a + (long)L.nr * (b + (long)L.nt * c);
                const float4 g0 = *reinterpret_cast<const float4 *>(dy + idx * cout + cg * 8);
                const float4 g1 = *reinterpret_cast<const float4 *>(dy + idx * cout + cg * 8 + 4);
                f[0] = g0.x; f[1] = g0.y; f[2] = g0.z; f[3] = g0.w; f[4] = g1.x; f[5] = g1.y; f[6] = g1.z; f[7] = g1.w;
                if (yout) {
                    const uint4 u = *reinterpret_cast<const uint4 *>(yout + idx * cout + cg * 8);
                    const bf16 *h = reinterpret_cast<const bf16 *>(&u);
#pragma unroll
                    for (int e = 0; e < 8; e++)
                        if (!(bf2f(h[e]) > 0.0f)) f[e] = 0.0f;
                }
            }
#pragma unroll
            for (int e = 0; e < 8; e += 2) {
                const unsigned pk = pack_bf16(f[e], f[e + 1]);
                dyT[(cg * 8 + e) * kWLdy + row * kTR + i] = (bf16)(pk & 0xFFFFu);
                dyT[(cg * 8 + e + 1) * kWLdy + row * kTR + i] = (bf16)(pk >> 16);
            }
        }
        // xsT[((di * 4 + hk) * 4 + hj) * 16 + ci][i] = x[r0 + i + di - 1][j0 + hj - 1][k0 + hk - 1][slice ci]
        for (int it = tid; it < 3 * 4 * 4 * kTR * 2; it += kTB) {
            const int i = it % kTR, h = (it / kTR) & 1, rest = it / (2 * kTR);
            const int hj = rest % 4, hk = (rest / 4) % 4, di = rest / 16;
            int a = r0 + i + di - 1, b = j0 + hj - 1, c = k0 + hk - 1;
            c = (c < 0) ? c + L.np : (c >= L.np ? c - L.np : c);
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if ((unsigned)a < (unsigned)L.nr && (unsigned)b < (unsigned)L.nt && (unsigned)c < (unsigned)L.np) {
                const int ch = sl * 16 + h * 8;
                if (ch < c1) {
                    const long e = up1 ? (a >> 1) + (long)cr * ((b >> 1) + (long)ct * (c >> 1))
                                       : a + (long)L.nr * (b + (long)L.nt * c);
                    v = *reinterpret_cast<const uint4 *>(x1 + e * c1 + ch);
                } else {
                    const long e = a + (long)L.nr * (b + (long)L.nt * c);
                    v = *reinterpret_cast<const uint4 *>(x2 + e * c2 + (ch - c1));
                }
            }
            const bf16 *hv = reinterpret_cast<const bf16 *>(&v);
            bf16 *dst = xsT + (((di * 4 + hk) * 4 + hj) * 16 + h * 8) * kWLx + i;
#pragma unroll
            for (int e = 0; e < 8; e++) dst[e * kWLx] = hv[e];
        }
        __syncthreads();
        // A fragments: co = t * 16 + lane % 16, cells row * 32 + 8 (lane / 16) .. + 7
        bf16x8 af[NTO][4];
#pragma unroll
        for (int t = 0; t < NTO; t++)
#pragma unroll
            for (int row = 0; row < 4; row++)
                af[t][row] = *reinterpret_cast<const bf16x8 *>(dyT + (t * 16 + (lane & 15)) * kWLdy + row * kTR +
                                                               8 * (lane >> 4));
#pragma unroll
        for (int q = 0; q < 7; q++) {
            const int tap = wv + 4 * q;
            if (tap < 27) {
                const int di = tap % 3, dj = (tap / 3) % 3, dk = tap / 9;  // each in 0..2 (offset + 1)
#pragma unroll
                for (int row = 0; row < 4; row++) {
                    const int hj = (row & 1) + dj, hk = (row >> 1) + dk;
                    const bf16x8 bfr = *reinterpret_cast<const bf16x8 *>(
                        xsT + (((di * 4 + hk) * 4 + hj) * 16 + (lane & 15)) * kWLx + 8 * (lane >> 4));
#pragma unroll
                    for (int t = 0; t < NTO; t++)
                        acc[q][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[t][row], bfr, acc[q][t], 0, 0, 0);
                }
            }
        }
    }
    // partial sums of this block: part[blockIdx.x][tap][co][ci]
#pragma unroll
    for (int q = 0; q < 7; q++) {
        const int tap = wv + 4 * q;
        if (tap < 27) {
            float *o = part + ((long)blockIdx.x * 27 + tap) * cout * cin + sl * 16 + (lane & 15);
#pragma unroll
            for (int t = 0; t < NTO; t++)
#pragma unroll
                for (int i = 0; i < 4; i++) o[(long)(t * 16 + 4 * (lane >> 4) + i) * cin] = acc[q][t][i];
        }
    }
}

// dw[w] = sum over chunks of part (fixed order, deterministic); nw = 27 Cout Cin.
__global__ __launch_bounds__(kTB) void k_sum_parts(long nw, int nchunk, const float *__restrict__ part,
                                                   float *__restrict__ dw)
{
    long w = (long)blockIdx.x * kTB + threadIdx.x;
    if (w >= nw) return;
    float s = 0.0f;
    for (int ch = 0; ch < nchunk; ch++) s += part[(long)ch * nw + w];
    dw[w] = s;
}

// Partial channel sums of the masked gradient (bias gradient): part[chunk][co].
__global__ __launch_bounds__(kTB) void k_bias_parts(long n, int cout, const float *__restrict__ dy,
                                                    const bf16 *__restrict__ yout, long chunk, float *__restrict__ part)
{
    __shared__ float sh[kTB];
    const int co = threadIdx.x % cout, g = threadIdx.x / cout, ng = kTB / cout;
    const long c0 = (long)blockIdx.x * chunk, c1 = c0 + chunk < n ? c0 + chunk : n;
    float s = 0.0f;
    if (g < ng)
        for (long c = c0 + g; c < c1; c += ng) {
            float v = dy[c * cout + co];
            if (yout && !(bf2f(yout[c * cout + co]) > 0.0f)) v = 0.0f;
            s += v;
        }
    sh[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < cout) {
        float t = 0.0f;
        for (int q = 0; q < ng; q++) t += sh[q * cout + threadIdx.x];
        part[(long)blockIdx.x * cout + threadIdx.x] = t;
    }
}

// ------------------------------------------------------- pooling / upsampling

// 2x2x2 average pooling (bf16 in / out, fp32 arithmetic, the 8 children summed in the
// order r, theta, phi); coarse level Lc.  A thread owns 8 channels of one coarse cell:
// eight 16-byte loads (the children, two by two adjacent in r) and one 16-byte store.
__global__ __launch_bounds__(kTB) void k_pool(Lv Lc, int C, const bf16 *__restrict__ x, bf16 *__restrict__ y)
{
    const int ng = C >> 3;
    const long idx = (long)blockIdx.x * kTB + threadIdx.x;
    if (idx >= Lc.n * ng) return;
    const long g = idx / ng;
    const int ch = (int)(idx - g * ng) * 8;
    int I, J, K;
    cell_coords(Lc, g, I, J, K);
    const long fr = 2 * Lc.nr, ft = 2 * Lc.nt;
    uint4 u[8];
#pragma unroll
    for (int q = 0; q < 8; q++) {
        const long f = (2 * I + (q & 1)) + fr * ((2 * J + ((q >> 1) & 1)) + ft * (2 * K + (q >> 2)));
        u[q] = *reinterpret_cast<const uint4 *>(x + f * C + ch);
    }
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 8; q++) {
        const unsigned wd[4] = {u[q].x, u[q].y, u[q].z, u[q].w};
#pragma unroll
        for (int e = 0; e < 8; e++) s[e] += bf2f((bf16)(e & 1 ? wd[e >> 1] >> 16 : wd[e >> 1] & 0xFFFFu));
    }
    unsigned o[4];
#pragma unroll
    for (int e = 0; e < 4; e++)
        o[e] = (unsigned)f2bf(s[2 * e] * 0.125f) | ((unsigned)f2bf(s[2 * e + 1] * 0.125f) << 16);
    *reinterpret_cast<uint4 *>(y + g * C + ch) = make_uint4(o[0], o[1], o[2], o[3]);
}

// dx_fine += dy_coarse / 8 (pooling adjoint), fine level Lf.
__global__ __launch_bounds__(kTB) void k_pool_bwd_add(Lv Lf, int C, const float *__restrict__ dyc, float *__restrict__ dxf)
{
    long idx = (long)blockIdx.x * kTB + threadIdx.x;
    if (idx >= Lf.n * C) return;
    const long f = idx / C;
    const int ch = (int)(idx % C);
    int i, j, k;
    cell_coords(Lf, f, i, j, k);
    const long g = (i >> 1) + (long)(Lf.nr >> 1) * ((j >> 1) + (long)(Lf.nt >> 1) * (k >> 1));
    dxf[idx] += dyc[g * C + ch] * 0.125f;
}

// dx_coarse[g] = sum of the 8 fine children of dy_fine (upsampling adjoint); coarse level Lc.
__global__ __launch_bounds__(kTB) void k_up_bwd(Lv Lc, int C, const float *__restrict__ dyf, float *__restrict__ dxc)
{
    long idx = (long)blockIdx.x * kTB + threadIdx.x;
    if (idx >= Lc.n * C) return;
    const long g = idx / C;
    const int ch = (int)(idx % C);
    int I, J, K;
    cell_coords(Lc, g, I, J, K);
    const int fr = 2 * Lc.nr, ft = 2 * Lc.nt;
    float s = 0.0f;
    for (int q = 0; q < 8; q++) {
        long f = (2 * I + (q & 1)) + (long)fr * ((2 * J + ((q >> 1) & 1)) + (long)ft * (2 * K + (q >> 2)));
        s += dyf[f * C + ch];
    }
    dxc[idx] = s;
}

// ------------------------------------------------------------- 1x1 output

// z = w . x + b over 16 channels (fp32 out).
__global__ __launch_bounds__(kTB) void k_out_fwd(long n, const bf16 *__restrict__ x, const bf16 *__restrict__ w,
                                                 const float *__restrict__ b, const double *__restrict__ scale,
                                                 float *__restrict__ z)
{
    long c = (long)blockIdx.x * kTB + threadIdx.x;
    if (c >= n) return;
    // the cell's 16 channels as two 16-byte loads
    const uint4 u0 = *reinterpret_cast<const uint4 *>(x + c * 16), u1 = *reinterpret_cast<const uint4 *>(x + c * 16 + 8);
    const unsigned wd[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
    float s = b[0];
#pragma unroll
    for (int q = 0; q < 16; q++) s = fmaf(bf2f(w[q]), bf2f((bf16)(q & 1 ? wd[q >> 1] >> 16 : wd[q >> 1] & 0xFFFFu)), s);
    // scale != nullptr: the preconditioner's output scaled back by scale[1] (the input was
    // scaled by scale[0] = 1 / scale[1]; the map is taken as positively homogeneous of
    // degree one)
    z[c] = scale ? (float)((double)s * scale[1]) : s;
}

// dx[c][q] = w[q] gz[c]; per-block partials of dw[q] = sum gz x[q] and db = sum gz.
__global__ __launch_bounds__(kTB) void k_out_bwd(long n, const bf16 *__restrict__ x, const bf16 *__restrict__ w,
                                                 const float *__restrict__ gz, float *__restrict__ dx, long chunk,
                                                 float *__restrict__ part)
{
    __shared__ float sh[kTB][17];
    const long c0 = (long)blockIdx.x * chunk, c1 = c0 + chunk < n ? c0 + chunk : n;
    float acc[17] = {0.0f};
    for (long c = c0 + threadIdx.x; c < c1; c += kTB) {
        const float g = gz[c];
        acc[16] += g;
#pragma unroll
        for (int q = 0; q < 16; q++) {
            acc[q] += g * bf2f(x[c * 16 + q]);
            dx[c * 16 + q] = bf2f(w[q]) * g;
        }
    }
#pragma unroll
    for (int q = 0; q < 17; q++) sh[threadIdx.x][q] = acc[q];
    __syncthreads();
    if (threadIdx.x < 17) {
        float s = 0.0f;
        for (int t = 0; t < kTB; t++) s += sh[t][threadIdx.x];
        part[(long)blockIdx.x * 17 + threadIdx.x] = s;
    }
}

// ----------------------------------------------------------- input features

// Operator features of the scaled system, written once per system into channels 1..3 of
// the network input X[c][16] (channels 4..15 zero): for each outward face, -ahat in
// log10, clipped to [-30, 0] and mapped to [-1, 1].
__global__ __launch_bounds__(kTB) void k_features(long n, const double *__restrict__ ahat, bf16 *__restrict__ X)
{
    long c = (long)blockIdx.x * kTB + threadIdx.x;
    if (c >= n) return;
    X[c * 16] = 0;
    for (int d = 0; d < 3; d++) {
        double a = -ahat[(long)d * n + c];
        double f = a > 1e-30 ? log10(a) : -30.0;
        f = f < -30.0 ? -30.0 : (f > 0.0 ? 0.0 : f);
        X[c * 16 + 1 + d] = f2bf((float)((f + 15.0) / 15.0));
    }
    for (int q = 4; q < 16; q++) X[c * 16 + q] = 0;
}

// Channel 0 of the network input: the residual scaled to unit RMS, r * s.
template <typename V>
__global__ __launch_bounds__(kTB) void k_set_input(long n, const V *__restrict__ r, const double *__restrict__ scale,
                                                   bf16 *__restrict__ X)
{
    long c = (long)blockIdx.x * kTB + threadIdx.x;
    if (c >= n) return;
    X[c * 16] = f2bf((float)((double)r[c] * scale[0]));
}

// ------------------------------------------------------------ loss, Adam

// Per-block partials of sum (z - e)^2 and sum e^2.
__global__ __launch_bounds__(kTB) void k_loss_parts(long n, const float *__restrict__ z, const float *__restrict__ e,
                                                    long chunk, double *__restrict__ part)
{
    __shared__ double sa[kTB], sb[kTB];
    const long c0 = (long)blockIdx.x * chunk, c1 = c0 + chunk < n ? c0 + chunk : n;
    double a = 0.0, b = 0.0;
    for (long c = c0 + threadIdx.x; c < c1; c += kTB) {
        double d = (double)z[c] - (double)e[c];
        a += d * d;
        b += (double)e[c] * (double)e[c];
    }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0, t = 0.0;
        for (int q = 0; q < kTB; q++) {
            s += sa[q];
            t += sb[q];
        }
        part[2 * blockIdx.x] = s;
        part[2 * blockIdx.x + 1] = t;
    }
}

// Sums the loss partials (thread 0, fixed order): res[0] = loss, res[1] = sum e^2.
__global__ void k_loss_finish(int nb, const double *__restrict__ part, double *__restrict__ res)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0, t = 0.0;
    for (int q = 0; q < nb; q++) {
        s += part[2 * q];
        t += part[2 * q + 1];
    }
    res[0] = t > 0.0 ? s / t : 0.0;
    res[1] = t;
}

// dL/dz = 2 (z - e) / sum e^2.
__global__ __launch_bounds__(kTB) void k_loss_grad(long n, const float *__restrict__ z, const float *__restrict__ e,
                                                   const double *__restrict__ res, float *__restrict__ gz)
{
    long c = (long)blockIdx.x * kTB + threadIdx.x;
    if (c >= n) return;
    gz[c] = (float)(2.0 * ((double)z[c] - (double)e[c]) / res[1]);
}

// Adam on the fp32 master parameters (bias-corrected), then the bf16 copies.
__global__ __launch_bounds__(kTB) void k_adam(long np_, float *__restrict__ p, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v, float lr, float b1,
                                              float b2, float eps, float c1, float c2)
{
    long i = (long)blockIdx.x * kTB + threadIdx.x;
    if (i >= np_) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// bf16 copies of one layer's weights: w [taps][cout][cin] and wt [taps][cin][cout].
__global__ __launch_bounds__(kTB) void k_cast_weights(int taps, int cout, int cin, const float *__restrict__ p,
                                                      bf16 *__restrict__ w, bf16 *__restrict__ wt)
{
    long i = (long)blockIdx.x * kTB + threadIdx.x;
    const long nw = (long)taps * cout * cin;
    if (i >= nw) return;
    const int ci = (int)(i % cin);
    const long r = i / cin;
    const int co = (int)(r % cout), t = (int)(r / cout);
    const bf16 h = f2bf(p[i]);
    w[i] = h;
    if (wt) wt[((long)t * cin + ci) * cout + co] = h;
}

// Training target: e = (y* - y) * scale (fp32).
__global__ __launch_bounds__(kTB) void k_pair_target(long n, const double *__restrict__ ystar, const double *__restrict__ y,
                                                     const double *__restrict__ scale, float *__restrict__ e)
{
    long c = (long)blockIdx.x * kTB + threadIdx.x;
    if (c < n) e[c] = (float)((ystar[c] - y[c]) * scale[0]);
}

// scale = sqrt(n / res2) from the residual norm of the last k_resid.
__global__ void k_pair_scale(long n, const DevScalars *sc, double *scale)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double r2 = sc->res2;
        double s = r2 > 0.0 ? sqrt((double)n / r2) : 1.0;
        scale[0] = s;
        scale[1] = 1.0 / s;
    }
}

// out = float(r * scale[0]): the scaled residual of a training pair in fp32.
__global__ __launch_bounds__(kTB) void k_scaled_f32(long n, const double *__restrict__ r,
                                                    const double *__restrict__ scale, float *__restrict__ out)
{
    long c = (long)blockIdx.x * kTB + threadIdx.x;
    if (c < n) out[c] = (float)(r[c] * scale[0]);
}

// fp32 -> bf16 and bf16 -> fp32 copies (tests, targets).
__global__ __launch_bounds__(kTB) void k_f2bf(long n, const float *__restrict__ x, bf16 *__restrict__ y)
{
    long i = (long)blockIdx.x * kTB + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

// ------------------------------------------------------------------ launchers

static unsigned nblk(long n) { return (unsigned)((n + kTB - 1) / kTB); }

// Persistent grid: as many blocks as fit on the 256 compute units at once (by LDS),
// but no more than there are tiles (rounded up to a multiple of 8).
template <int TJ, int TK>
unsigned conv_grid(const Lv &L, const void *kernel, size_t lds)
{
    const long ntiles = (long)((L.nr + kTR - 1) / kTR) * ((L.nt + TJ - 1) / TJ) * ((L.np + TK - 1) / TK);
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, kTB, lds) != hipSuccess || occ < 1) occ = 1;
    const long per_cu = occ;
    const long g = std::min<long>(256 * per_cu, (ntiles + 7) / 8 * 8);
    return (unsigned)std::max<long>(8, g);
}

template <int NT, int TJ, int TK>
void launch_fwd_t(const Lv &L, const bf16 *x1, int c1, int up1, const bf16 *x2, int c2, const bf16 *w, const float *b,
                  int relu, bf16 *y, float *yf, hipStream_t s)
{
    constexpr size_t lds = conv_lds_bytes<NT, TJ, TK>();
    static const bool attr = hipFuncSetAttribute((const void *)k_conv_fwd<NT, TJ, TK>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess;
    (void)attr;
    hipLaunchKernelGGL((k_conv_fwd<NT, TJ, TK>), dim3(conv_grid<TJ, TK>(L, (const void *)k_conv_fwd<NT, TJ, TK>, lds)), dim3(kTB), lds, s, L, x1, c1, up1, x2,
                       c2, w, b, relu, y, yf);
}

// One block per (theta tile, r tile, phi chunk) of conv_slide, rounded up to a multiple of 8.
unsigned slide_grid(const Lv &L)
{
    const long n = (long)((L.nr + kTR - 1) / kTR) * ((L.nt + kSlideTJ - 1) / kSlideTJ) *
                   ((L.np + kSlideP - 1) / kSlideP);
    return (unsigned)((n + 7) / 8 * 8);
}

void launch_fwd_slide(const Lv &L, const bf16 *x1, int c1, int up1, const bf16 *x2, int c2, const bf16 *w,
                      const float *b, int relu, bf16 *y, float *yf, hipStream_t s)
{
    constexpr size_t lds = slide_lds_bytes<kSlideTJ>();
    static const bool attr = hipFuncSetAttribute((const void *)k_conv_fwd<1, kSlideTJ, 1, true>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess;
    (void)attr;
    hipLaunchKernelGGL((k_conv_fwd<1, kSlideTJ, 1, true>), dim3(slide_grid(L)), dim3(kTB), lds, s, L, x1, c1, up1, x2,
                       c2, w, b, relu, y, yf);
}

void launch_conv_fwd_pool(const Lv &L, const bf16 *x, const bf16 *w, const float *b, bf16 *y, bf16 *yp, hipStream_t s)
{
    constexpr size_t lds = slide_lds_bytes<kSlideTJ>();
    static const bool attr = hipFuncSetAttribute((const void *)k_conv_fwd_pool, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds) == hipSuccess;
    (void)attr;
    hipLaunchKernelGGL(k_conv_fwd_pool, dim3(slide_grid(L)), dim3(kTB), lds, s, L, x, w, b, y, yp);
}

void launch_conv_fwd_head(const Lv &L, const bf16 *x, const bf16 *w, const float *b, const bf16 *wo, const float *bo,
                          const double *scale, float *z, hipStream_t s)
{
    constexpr size_t lds = slide_lds_bytes<kSlideTJ>();
    static const bool attr = hipFuncSetAttribute((const void *)k_conv_fwd_head, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds) == hipSuccess;
    (void)attr;
    hipLaunchKernelGGL(k_conv_fwd_head, dim3(slide_grid(L)), dim3(kTB), lds, s, L, x, w, b, wo, bo, scale, z);
}

// One block per (theta tile, r tile, phi chunk) of k_conv_fwd_dec, rounded up to a
// multiple of 8 (the fine level's dimensions are even: it has a coarser level).
void launch_fwd_dec(const Lv &L, const bf16 *x1, const bf16 *x2, const bf16 *w, const float *b, int relu, bf16 *y,
                    float *yf, hipStream_t s)
{
    constexpr size_t lds = DecGeom::lds;
    static const bool attr = hipFuncSetAttribute((const void *)k_conv_fwd_dec, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds) == hipSuccess;
    (void)attr;
    const long n = (long)((L.nr + kTR - 1) / kTR) * ((L.nt + kDecTJ - 1) / kDecTJ) * ((L.np + kSlideP - 1) / kSlideP);
    hipLaunchKernelGGL(k_conv_fwd_dec, dim3((unsigned)((n + 7) / 8 * 8)), dim3(kDecTB), lds, s, L, x1, x2, w, b, relu,
                       y, yf);
}

template <int NT, int TJ, int TK>
void launch_bwd_t(const Lv &L, const float *dy, const bf16 *y, int cout, const bf16 *wt, int c1, float *d1, int c2,
                  float *d2, hipStream_t s)
{
    constexpr size_t lds = conv_lds_bytes<NT, TJ, TK>();
    static const bool attr = hipFuncSetAttribute((const void *)k_conv_bwd_data<NT, TJ, TK>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess;
    (void)attr;
    hipLaunchKernelGGL((k_conv_bwd_data<NT, TJ, TK>), dim3(conv_grid<TJ, TK>(L, (const void *)k_conv_bwd_data<NT, TJ, TK>, lds)), dim3(kTB), lds, s, L, dy, y,
                       cout, wt, c1, d1, c2, d2);
}

// Output-channel tiles NT = cout / 16; the theta x phi extent of a block's tile
// shrinks as NT grows so that accumulators and LDS stay within budget.
bool launch_conv_fwd(const Lv &L, const bf16 *x1, int c1, int up1, const bf16 *x2, int c2, const bf16 *w,
                     const float *b, int cout, int relu, bf16 *y, float *yf, hipStream_t s)
{
    if ((c1 + c2) % 16 || c1 % 16) return false;
    switch (cout) {
    case 16:
        if (c1 + c2 == 16) launch_fwd_slide(L, x1, c1, up1, x2, c2, w, b, relu, y, yf, s);
        else if (up1 && c1 == 32 && c2 == 16) launch_fwd_dec(L, x1, x2, w, b, relu, y, yf, s);
        else launch_fwd_t<1, 4, 4>(L, x1, c1, up1, x2, c2, w, b, relu, y, yf, s);
        return true;
    case 32: launch_fwd_t<2, 4, 4>(L, x1, c1, up1, x2, c2, w, b, relu, y, yf, s); return true;
    case 48: launch_fwd_t<3, 4, 2>(L, x1, c1, up1, x2, c2, w, b, relu, y, yf, s); return true;
    case 64: launch_fwd_t<4, 4, 2>(L, x1, c1, up1, x2, c2, w, b, relu, y, yf, s); return true;
    default: return false;
    }
}

bool launch_conv_bwd_data(const Lv &L, const float *dy, const bf16 *y, int cout, const bf16 *wt, int c1, float *d1,
                          int c2, float *d2, hipStream_t s)
{
    if (cout % 16 || c1 % 16) return false;
    switch ((c1 + c2) / 16) {
    case 1: launch_bwd_t<1, 4, 4>(L, dy, y, cout, wt, c1, d1, c2, d2, s); return true;
    case 2: launch_bwd_t<2, 4, 4>(L, dy, y, cout, wt, c1, d1, c2, d2, s); return true;
    case 3: launch_bwd_t<3, 4, 2>(L, dy, y, cout, wt, c1, d1, c2, d2, s); return true;
    case 4: launch_bwd_t<4, 4, 2>(L, dy, y, cout, wt, c1, d1, c2, d2, s); return true;
    case 6: launch_bwd_t<6, 2, 2>(L, dy, y, cout, wt, c1, d1, c2, d2, s); return true;
    default: return false;
    }
}

// Weight and bias gradients of one 3x3x3 layer: dw (27 Cout Cin), db (Cout); part holds
// ceil(n / 2048) * 27 * Cout * Cin floats.
// Blocks per input slice of the weight-gradient kernel (the number of partial sums).
long wgrad_blocks(const Lv &L)
{
    const long ntiles = (long)((L.nr + kTR - 1) / kTR) * ((L.nt + 1) / 2) * ((L.np + 1) / 2);
    return std::min<long>(256, ntiles);
}

// Floats of the partial-sum buffer one weight gradient needs (the bias partials fit too).
long wgrad_part_floats(const Lv &L, int cout, int cin)
{
    const long nw = 27L * cout * cin;
    return std::max<long>(wgrad_blocks(L) * nw, ((L.n + 2047) / 2048) * cout);
}

template <int NTO>
void launch_wgrad_t(const Lv &L, const float *dy, const bf16 *y, const bf16 *x1, int c1, int up1, const bf16 *x2,
                    int c2, float *part, hipStream_t s)
{
    constexpr size_t lds = wgrad_lds_bytes<NTO>();
    static const bool attr = hipFuncSetAttribute((const void *)k_conv_wgrad<NTO>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess;
    (void)attr;
    hipLaunchKernelGGL(k_conv_wgrad<NTO>, dim3((unsigned)wgrad_blocks(L), (unsigned)((c1 + c2) / 16)), dim3(kTB), lds, s,
                       L, dy, y, x1, c1, up1, x2, c2, part);
}

// Weight and bias gradients of one 3x3x3 layer: dw (27 Cout Cin), db (Cout); part holds
// wgrad_part_floats(L, cout, c1 + c2) floats.
bool launch_conv_bwd_weight(const Lv &L, const float *dy, const bf16 *y, int cout, const bf16 *x1, int c1, int up1,
                            const bf16 *x2, int c2, float *part, float *dw, float *db, hipStream_t s)
{
    if ((c1 + c2) % 16 || c1 % 16) return false;
    switch (cout) {
    case 16: launch_wgrad_t<1>(L, dy, y, x1, c1, up1, x2, c2, part, s); break;
    case 32: launch_wgrad_t<2>(L, dy, y, x1, c1, up1, x2, c2, part, s); break;
    case 48: launch_wgrad_t<3>(L, dy, y, x1, c1, up1, x2, c2, part, s); break;
    case 64: launch_wgrad_t<4>(L, dy, y, x1, c1, up1, x2, c2, part, s); break;
    default: return false;
    }
    const long nw = 27L * cout * (c1 + c2);
    hipLaunchKernelGGL(k_sum_parts, dim3(nblk(nw)), dim3(kTB), 0, s, nw, (int)wgrad_blocks(L), part, dw);
    const long chunk = 2048;
    const int nc = (int)((L.n + chunk - 1) / chunk);
    hipLaunchKernelGGL(k_bias_parts, dim3(nc), dim3(kTB), 0, s, L.n, cout, dy, y, chunk, part);
    hipLaunchKernelGGL(k_sum_parts, dim3(nblk(cout)), dim3(kTB), 0, s, (long)cout, nc, part, db);
    return true;
}

void launch_pool(const Lv &Lc, int C, const bf16 *x, bf16 *y, hipStream_t s)
{
    hipLaunchKernelGGL(k_pool, dim3(nblk(Lc.n * (C / 8))), dim3(kTB), 0, s, Lc, C, x, y);  // C = 16 or 32
}

void launch_pool_bwd_add(const Lv &Lf, int C, const float *dyc, float *dxf, hipStream_t s)
{
    hipLaunchKernelGGL(k_pool_bwd_add, dim3(nblk(Lf.n * C)), dim3(kTB), 0, s, Lf, C, dyc, dxf);
}

void launch_up_bwd(const Lv &Lc, int C, const float *dyf, float *dxc, hipStream_t s)
{
    hipLaunchKernelGGL(k_up_bwd, dim3(nblk(Lc.n * C)), dim3(kTB), 0, s, Lc, C, dyf, dxc);
}

void launch_out_fwd(long n, const bf16 *x, const bf16 *w, const float *b, const double *scale, float *z,
                    hipStream_t s)
{
    hipLaunchKernelGGL(k_out_fwd, dim3(nblk(n)), dim3(kTB), 0, s, n, x, w, b, scale, z);
}

void launch_conv_fwd_in(const Lv &L, const bf16 *X, const float *r, const double *scale, const bf16 *w,
                        const float *b, bf16 *y, hipStream_t s)
{
    constexpr size_t lds = slide_lds_bytes<kSlideTJ>();
    static const bool attr = hipFuncSetAttribute((const void *)k_conv_fwd_in<true>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess;
    (void)attr;
    hipLaunchKernelGGL(k_conv_fwd_in<true>, dim3(slide_grid(L)), dim3(kTB), lds, s, L, X, r, scale, w, b, y);
}

// 1x1 output layer backward: dx, and dw[16], db into dwb[17]; part holds ceil(n/2048)*17.
void launch_out_bwd(long n, const bf16 *x, const bf16 *w, const float *gz, float *dx, float *part, float *dwb,
                    hipStream_t s)
{
    const long chunk = 2048;
    const int nc = (int)((n + chunk - 1) / chunk);
    hipLaunchKernelGGL(k_out_bwd, dim3(nc), dim3(kTB), 0, s, n, x, w, gz, dx, chunk, part);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kTB), 0, s, 17L, nc, part, dwb);
}

void launch_features(long n, const double *ahat, bf16 *X, hipStream_t s)
{
    hipLaunchKernelGGL(k_features, dim3(nblk(n)), dim3(kTB), 0, s, n, ahat, X);
}

void launch_set_input(long n, const double *r, const double *scale, bf16 *X, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_input<double>, dim3(nblk(n)), dim3(kTB), 0, s, n, r, scale, X);
}

// loss into res[0] (and sum e^2 into res[1]) and dL/dz into gz; part holds 2 * 4096 doubles.
void launch_loss(long n, const float *z, const float *e, double *part, double *res, float *gz, hipStream_t s)
{
    long chunk = n > 4096L * 4096L ? (n + 4095) / 4096 : 4096;
    int nb = (int)((n + chunk - 1) / chunk);
    hipLaunchKernelGGL(k_loss_parts, dim3(nb), dim3(kTB), 0, s, n, z, e, chunk, part);
    hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(64), 0, s, nb, part, res);
    if (gz) hipLaunchKernelGGL(k_loss_grad, dim3(nblk(n)), dim3(kTB), 0, s, n, z, e, res, gz);
}

void launch_adam(long np_, float *p, const float *g, float *m, float *v, float lr, float b1, float b2, float eps,
                 float c1, float c2, hipStream_t s)
{
    hipLaunchKernelGGL(k_adam, dim3(nblk(np_)), dim3(kTB), 0, s, np_, p, g, m, v, lr, b1, b2, eps, c1, c2);
}

void launch_cast_weights(int taps, int cout, int cin, const float *p, bf16 *w, bf16 *wt, hipStream_t s)
{
    hipLaunchKernelGGL(k_cast_weights, dim3(nblk((long)taps * cout * cin)), dim3(kTB), 0, s, taps, cout, cin, p, w, wt);
}

void launch_scaled_f32(long n, const double *r, const double *scale, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_scaled_f32, dim3(nblk(n)), dim3(kTB), 0, s, n, r, scale, out);
}

void launch_pair(long n, const DevScalars *sc, const double *ystar, const double *y, double *scale, float *e,
                 hipStream_t s)
{
    hipLaunchKernelGGL(k_pair_scale, dim3(1), dim3(64), 0, s, n, sc, scale);
    hipLaunchKernelGGL(k_pair_target, dim3(nblk(n)), dim3(kTB), 0, s, n, ystar, y, scale, e);
}

}  // namespace nn
}  // namespace rt
