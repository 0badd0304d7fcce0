// Kernels of the learned preconditioner: a 3-level 3-D convolutional U-Net (3x3x3
// kernels, 16/32/64 channels) evaluated and trained in BF16 on the matrix cores with
// FP32 accumulation.
//
// Tensors are channels-last, x[c * C + ch], on the spherical grid levels (cell
// c = i + nr (j + nt k)); convolutions pad with zeros in r and theta and wrap in phi.
// Tap t = (dk+1) 9 + (dj+1) 3 + (di+1); weights w[(t Cout + co) Cin + ci] (and a
// transposed copy wt[(t Cin + ci) Cout + co] for the data gradient).
//
// Every 3x3x3 convolution is an implicit GEMM on v_mfma_f32_16x16x16_bf16: a wavefront
// owns 16 cells (the M dimension) and all output channels (N, 16 per MFMA tile); K runs
// over the 27 taps times the input channels in chunks of 16.  Lane l supplies
// A[m = l%16][k = 4(l/16) .. +3] (4 consecutive channels of its cell's neighbour: one
// 8-byte load in the channels-last layout), B[k = 4(l/16) .. +3][n = l%16] (4
// consecutive input channels of one output channel's weights: one 8-byte load), and
// receives D[m = 4(l/16) .. +3][n = l%16].  A decoder convolution reads two sources
// (the nearest-neighbour upsampled coarse tensor and the skip tensor) directly, so the
// upsampled/concatenated tensor is never materialised.
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

// ------------------------------------------------------------- forward conv

// y = act(conv([up?(x1), x2], w) + bias) with NT * 16 output channels.  x1 has c1
// channels and lives on the level of y (up1 = 0) or on the next coarser level
// (up1 = 1, read through nearest-neighbour upsampling); x2 (c2 channels, may be 0) on
// the level of y.  Writes bf16 y and/or fp32 yf.
template <int NT>
__global__ __launch_bounds__(kTB) void k_conv_fwd(Lv L, const bf16 *__restrict__ x1, int c1, int up1,
                                                  const bf16 *__restrict__ x2, int c2, const bf16 *__restrict__ w,
                                                  const float *__restrict__ bias, int relu, bf16 *__restrict__ y,
                                                  float *__restrict__ yf)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long cell0 = ((long)blockIdx.x * (kTB / 64) + wv) * 16;
    if (cell0 >= L.n) return;
    const int m = lane & 15, kq = lane >> 4;
    long cm = cell0 + m;
    if (cm >= L.n) cm = L.n - 1;
    int i, j, k;
    cell_coords(L, cm, i, j, k);
    const int cin = c1 + c2, cout = NT * 16;
    const int cr = L.nr >> 1, ct = L.nt >> 1;
    float4v acc[NT];
#pragma unroll
    for (int t = 0; t < NT; t++) acc[t] = float4v{0.f, 0.f, 0.f, 0.f};
    for (int tap = 0; tap < 27; tap++) {
        int a, b, c;
        const bool ok = tap_nb(L, i, j, k, tap, 1, a, b, c);
        const long e = ok ? a + (long)L.nr * (b + (long)L.nt * c) : cm;
        const long e1 = up1 ? (ok ? (a >> 1) + (long)cr * ((b >> 1) + (long)ct * (c >> 1)) : 0) : e;
        const bf16 *wt = w + (long)tap * cout * cin;
        for (int c0 = 0; c0 < cin; c0 += 16) {
            const short4v av = (c0 < c1) ? ld4(x1 + e1 * c1 + c0 + 4 * kq, ok)
                                         : ld4(x2 + e * c2 + (c0 - c1) + 4 * kq, ok);
#pragma unroll
            for (int t = 0; t < NT; t++) {
                const short4v bv = ld4(wt + (long)(t * 16 + m) * cin + c0 + 4 * kq, true);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[t], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NT; t++) {
        const float bb = bias ? bias[t * 16 + m] : 0.0f;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const long cell = cell0 + 4 * kq + r;
            if (cell < L.n) {
                float v = acc[t][r] + bb;
                if (relu && v < 0.0f) v = 0.0f;
                const long o = cell * cout + t * 16 + m;
                if (y) y[o] = f2bf(v);
                if (yf) yf[o] = v;
            }
        }
    }
}

// --------------------------------------------------------- data gradient

// dX = conv^T(dYm, w) for the concatenated input [up?(x1), x2] of a convolution with
// cout output channels (dYm = dY masked by the layer's ReLU output y when y != 0).
// Output at the level of dY, NTI * 16 input channels: channels < c1 to d1 ([n][c1];
// for an upsampled x1 this is the gradient of the upsampled tensor, folded onto the
// coarse level by k_up_bwd), the rest to d2 ([n][c2]).  Uses the transposed weights.
template <int NTI>
__global__ __launch_bounds__(kTB) void k_conv_bwd_data(Lv L, const float *__restrict__ dy, const bf16 *__restrict__ yout,
                                                       int cout, const bf16 *__restrict__ wt, int c1,
                                                       float *__restrict__ d1, int c2, float *__restrict__ d2)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long cell0 = ((long)blockIdx.x * (kTB / 64) + wv) * 16;
    if (cell0 >= L.n) return;
    const int m = lane & 15, kq = lane >> 4;
    long cm = cell0 + m;
    if (cm >= L.n) cm = L.n - 1;
    int i, j, k;
    cell_coords(L, cm, i, j, k);
    const int cin = c1 + c2;
    float4v acc[NTI];
#pragma unroll
    for (int t = 0; t < NTI; t++) acc[t] = float4v{0.f, 0.f, 0.f, 0.f};
    for (int tap = 0; tap < 27; tap++) {
        int a, b, c;
        const bool ok = tap_nb(L, i, j, k, tap, -1, a, b, c);  // output cell whose tap reads this cell
        const long o = ok ? a + (long)L.nr * (b + (long)L.nt * c) : cm;
        const bf16 *wtt = wt + (long)tap * cin * cout;
        for (int c0 = 0; c0 < cout; c0 += 16) {
            const short4v av = ld4_grad(dy + o * cout + c0 + 4 * kq, yout ? yout + o * cout + c0 + 4 * kq : nullptr, ok);
#pragma unroll
            for (int t = 0; t < NTI; t++) {
                const short4v bv = ld4(wtt + (long)(t * 16 + m) * cout + c0 + 4 * kq, true);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[t], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NTI; t++) {
        const int ci = t * 16 + m;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const long cell = cell0 + 4 * kq + r;
            if (cell < L.n) {
                if (ci < c1) d1[cell * c1 + ci] = acc[t][r];
                else d2[cell * c2 + (ci - c1)] = acc[t][r];
            }
        }
    }
}

// -------------------------------------------------------- weight gradient

// Partial dW over one chunk of cells and one tap: part[(chunk * 27 + tap) Cout Cin]
// = sum_{cells} dYm[cell][co] x[nb(cell, tap)][ci], as MFMA tiles with M = co,
// N = ci and K = cells (16 per MFMA).  Block: 4 wavefronts sharing the (co, ci) tile
// pairs; chunk = blockIdx.x, tap = blockIdx.y.
__global__ __launch_bounds__(kTB) void k_conv_bwd_weight(Lv L, const float *__restrict__ dy, const bf16 *__restrict__ yout,
                                                         int cout, const bf16 *__restrict__ x1, int c1, int up1,
                                                         const bf16 *__restrict__ x2, int c2, long chunk,
                                                         float *__restrict__ part)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int tap = blockIdx.y;
    const int cin = c1 + c2;
    const int nco = cout / 16, nci = cin / 16, npair = nco * nci;
    const long c_begin = (long)blockIdx.x * chunk;
    const long c_end = c_begin + chunk < L.n ? c_begin + chunk : L.n;
    const int cr = L.nr >> 1, ct = L.nt >> 1;
    float *out = part + ((long)blockIdx.x * 27 + tap) * cout * cin;
    for (int pr0 = wv; pr0 < npair; pr0 += 4 * 4) {
        // up to 4 tile pairs per pass per wavefront: pairs pr0, pr0+4, pr0+8, pr0+12
        float4v acc[4];
#pragma unroll
        for (int q = 0; q < 4; q++) acc[q] = float4v{0.f, 0.f, 0.f, 0.f};
        for (long cb = c_begin; cb < c_end; cb += 16) {
            // the four cells of this lane's K slice
            long cells[4];
            bool okc[4], okn[4];
            long e[4], e1[4];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                long cc = cb + 4 * kq + q;
                okc[q] = cc < c_end;
                cells[q] = okc[q] ? cc : c_begin;
                int i, j, k, a, b, c;
                cell_coords(L, cells[q], i, j, k);
                okn[q] = tap_nb(L, i, j, k, tap, 1, a, b, c) && okc[q];
                e[q] = okn[q] ? a + (long)L.nr * (b + (long)L.nt * c) : cells[q];
                e1[q] = up1 ? (okn[q] ? (a >> 1) + (long)cr * ((b >> 1) + (long)ct * (c >> 1)) : 0) : e[q];
            }
#pragma unroll
            for (int q4 = 0; q4 < 4; q4++) {
                const int pr = pr0 + 4 * q4;
                if (pr >= npair) break;
                const int ti = pr / nci, tj = pr % nci;  // co tile, ci tile
                const int co = ti * 16 + m, ci = tj * 16 + m;
                short4v av, bv;
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    float g = okc[q] ? dy[cells[q] * cout + co] : 0.0f;
                    if (yout && !(bf2f(yout[cells[q] * cout + co]) > 0.0f)) g = 0.0f;
                    av[q] = (short)f2bf(g);
                    bf16 xv = 0;
                    if (okn[q]) xv = (ci < c1) ? x1[e1[q] * c1 + ci] : x2[e[q] * c2 + (ci - c1)];
                    bv[q] = (short)xv;
                }
                acc[q4] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[q4], 0, 0, 0);
            }
        }
#pragma unroll
        for (int q4 = 0; q4 < 4; q4++) {
            const int pr = pr0 + 4 * q4;
            if (pr >= npair) break;
            const int ti = pr / nci, tj = pr % nci;
#pragma unroll
            for (int r = 0; r < 4; r++) out[(long)(ti * 16 + 4 * kq + r) * cin + tj * 16 + m] = acc[q4][r];
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

// 2x2x2 average pooling (bf16 in / out, fp32 arithmetic); coarse level Lc.
__global__ __launch_bounds__(kTB) void k_pool(Lv Lc, int C, const bf16 *__restrict__ x, bf16 *__restrict__ y)
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
        s += bf2f(x[f * C + ch]);
    }
    y[idx] = f2bf(s * 0.125f);
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
                                                 const float *__restrict__ b, float *__restrict__ z)
{
    long c = (long)blockIdx.x * kTB + threadIdx.x;
    if (c >= n) return;
    float s = b[0];
#pragma unroll
    for (int q = 0; q < 16; q++) s += bf2f(w[q]) * bf2f(x[c * 16 + q]);
    z[c] = s;
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

// fp32 -> bf16 and bf16 -> fp32 copies (tests, targets).
__global__ __launch_bounds__(kTB) void k_f2bf(long n, const float *__restrict__ x, bf16 *__restrict__ y)
{
    long i = (long)blockIdx.x * kTB + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

// ------------------------------------------------------------------ launchers

static unsigned nblk(long n) { return (unsigned)((n + kTB - 1) / kTB); }

bool launch_conv_fwd(const Lv &L, const bf16 *x1, int c1, int up1, const bf16 *x2, int c2, const bf16 *w,
                     const float *b, int cout, int relu, bf16 *y, float *yf, hipStream_t s)
{
    const unsigned nb = (unsigned)((L.n + 63) / 64);
    switch (cout) {
    case 16: hipLaunchKernelGGL(k_conv_fwd<1>, dim3(nb), dim3(kTB), 0, s, L, x1, c1, up1, x2, c2, w, b, relu, y, yf); return true;
    case 32: hipLaunchKernelGGL(k_conv_fwd<2>, dim3(nb), dim3(kTB), 0, s, L, x1, c1, up1, x2, c2, w, b, relu, y, yf); return true;
    case 48: hipLaunchKernelGGL(k_conv_fwd<3>, dim3(nb), dim3(kTB), 0, s, L, x1, c1, up1, x2, c2, w, b, relu, y, yf); return true;
    case 64: hipLaunchKernelGGL(k_conv_fwd<4>, dim3(nb), dim3(kTB), 0, s, L, x1, c1, up1, x2, c2, w, b, relu, y, yf); return true;
    default: return false;
    }
}

bool launch_conv_bwd_data(const Lv &L, const float *dy, const bf16 *y, int cout, const bf16 *wt, int c1, float *d1,
                          int c2, float *d2, hipStream_t s)
{
    const unsigned nb = (unsigned)((L.n + 63) / 64);
    switch ((c1 + c2) / 16) {
    case 1: hipLaunchKernelGGL(k_conv_bwd_data<1>, dim3(nb), dim3(kTB), 0, s, L, dy, y, cout, wt, c1, d1, c2, d2); return true;
    case 2: hipLaunchKernelGGL(k_conv_bwd_data<2>, dim3(nb), dim3(kTB), 0, s, L, dy, y, cout, wt, c1, d1, c2, d2); return true;
    case 3: hipLaunchKernelGGL(k_conv_bwd_data<3>, dim3(nb), dim3(kTB), 0, s, L, dy, y, cout, wt, c1, d1, c2, d2); return true;
    case 4: hipLaunchKernelGGL(k_conv_bwd_data<4>, dim3(nb), dim3(kTB), 0, s, L, dy, y, cout, wt, c1, d1, c2, d2); return true;
    case 6: hipLaunchKernelGGL(k_conv_bwd_data<6>, dim3(nb), dim3(kTB), 0, s, L, dy, y, cout, wt, c1, d1, c2, d2); return true;
    default: return false;
    }
}

// Weight and bias gradients of one 3x3x3 layer: dw (27 Cout Cin), db (Cout); part holds
// ceil(n / 2048) * 27 * Cout * Cin floats.
void launch_conv_bwd_weight(const Lv &L, const float *dy, const bf16 *y, int cout, const bf16 *x1, int c1, int up1,
                            const bf16 *x2, int c2, float *part, float *dw, float *db, hipStream_t s)
{
    const long chunk = 2048;
    const int nc = (int)((L.n + chunk - 1) / chunk);
    hipLaunchKernelGGL(k_conv_bwd_weight, dim3(nc, 27), dim3(kTB), 0, s, L, dy, y, cout, x1, c1, up1, x2, c2, chunk,
                       part);
    const long nw = 27L * cout * (c1 + c2);
    hipLaunchKernelGGL(k_sum_parts, dim3(nblk(nw)), dim3(kTB), 0, s, nw, nc, part, dw);
    hipLaunchKernelGGL(k_bias_parts, dim3(nc), dim3(kTB), 0, s, L.n, cout, dy, y, chunk, part);
    hipLaunchKernelGGL(k_sum_parts, dim3(nblk(cout)), dim3(kTB), 0, s, (long)cout, nc, part, db);
}

void launch_pool(const Lv &Lc, int C, const bf16 *x, bf16 *y, hipStream_t s)
{
    hipLaunchKernelGGL(k_pool, dim3(nblk(Lc.n * C)), dim3(kTB), 0, s, Lc, C, x, y);
}

void launch_pool_bwd_add(const Lv &Lf, int C, const float *dyc, float *dxf, hipStream_t s)
{
    hipLaunchKernelGGL(k_pool_bwd_add, dim3(nblk(Lf.n * C)), dim3(kTB), 0, s, Lf, C, dyc, dxf);
}

void launch_up_bwd(const Lv &Lc, int C, const float *dyf, float *dxc, hipStream_t s)
{
    hipLaunchKernelGGL(k_up_bwd, dim3(nblk(Lc.n * C)), dim3(kTB), 0, s, Lc, C, dyf, dxc);
}

void launch_out_fwd(long n, const bf16 *x, const bf16 *w, const float *b, float *z, hipStream_t s)
{
    hipLaunchKernelGGL(k_out_fwd, dim3(nblk(n)), dim3(kTB), 0, s, n, x, w, b, z);
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

void launch_set_input(long n, const float *r, const double *scale, bf16 *X, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_input<float>, dim3(nblk(n)), dim3(kTB), 0, s, n, r, scale, X);
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

void launch_pair(long n, const DevScalars *sc, const double *ystar, const double *y, double *scale, float *e,
                 hipStream_t s)
{
    hipLaunchKernelGGL(k_pair_scale, dim3(1), dim3(64), 0, s, n, sc, scale);
    hipLaunchKernelGGL(k_pair_target, dim3(nblk(n)), dim3(kTB), 0, s, n, ystar, y, scale, e);
}

}  // namespace nn
}  // namespace rt
