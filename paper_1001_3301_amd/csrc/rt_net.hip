// Host side of the learned preconditioner: the U-Net object (fp32 master weights,
// bf16 copies, Adam moments), its per-grid workspace, the forward / backward sequence,
// the training set built from the float64 method's own CG iterates, the training
// loop, and the layer-level C-ABI entry points.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "rt_internal.h"

using namespace rt;
using nn::bf16;
using nn::Lv;

namespace {

constexpr int NL = 11;
// layer: input channels (sum of sources), output channels, level (0 full, 1 half, 2 quarter)
const int CIN[NL] = {16, 16, 16, 32, 32, 64, 96, 32, 48, 16, 16};
const int COUT[NL] = {16, 16, 32, 32, 64, 64, 32, 32, 16, 16, 1};
const int LEVEL[NL] = {0, 0, 1, 1, 2, 2, 1, 1, 0, 0, 0};
int taps(int l) { return l == NL - 1 ? 1 : 27; }
long wcount(int l) { return (long)taps(l) * COUT[l] * CIN[l]; }
long poff(int l)
{
    long o = 0;
    for (int m = 0; m < l; m++) o += wcount(m) + COUT[m];
    return o;
}
constexpr int kTB = 256;
unsigned nblocks(long n) { return (unsigned)((n + kTB - 1) / kTB); }

thread_local std::string g_nerr;

}  // namespace

struct rt_net {
    int device = 0;
    long np_ = 0;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    bf16 *wb = nullptr, *wt = nullptr;
    int adam_t = 0;
    std::vector<void *> allocs;
    // workspace of one grid
    int nr = 0, nt = 0, nph = 0;
    bool train_ws = false;
    std::vector<void *> ws;
    Lv lv[3]{};
    bf16 *X = nullptr, *a[10] = {}, *p1 = nullptr, *p2 = nullptr;
    float *z = nullptr, *zin = nullptr;
    float *rq = nullptr, *gq = nullptr;  // residual loss: A z and dL/d(A z)
    float *g9, *g8, *gU8, *gS1, *g7, *g6, *gU6, *gS2, *g5, *g4, *gp2, *g2, *gp1, *g0, *gz;
    float *part = nullptr;
    size_t part_cap = 0;
    double *lpart = nullptr, *lres = nullptr, *scale = nullptr;
    std::string err;
};

struct rt_dataset {
    long n = 0;
    int cap = 0, size = 0;
    int nr = 0, nt = 0, nph = 0;
    bf16 *X = nullptr;    // [cap][n][16]
    float *E = nullptr;   // [cap][n] scaled errors e_k
    float *R = nullptr;   // [cap][n] scaled residuals r_k (fp32)
    float *A32 = nullptr; // [cap][3n] scaled operator of each added system
    std::vector<int> field;  // pair -> its system in A32
    int nfield = 0;
    double *ystar = nullptr, *y0 = nullptr;
    std::vector<void *> allocs;
};

namespace {

rt_status nfail(rt_net *net, rt_status s, const std::string &m)
{
    if (net) net->err = m;
    g_nerr = m;
    return s;
}

#define NN_HIP(net, call)                                                                            \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) return nfail((net), RT_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <class T>
T *nalloc(std::vector<void *> &list, size_t n)
{
    void *ptr = nullptr;
    if (hipMalloc(&ptr, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return nullptr;
    list.push_back(ptr);
    return static_cast<T *>(ptr);
}

void free_list(std::vector<void *> &l)
{
    for (void *ptr : l) (void)hipFree(ptr);
    l.clear();
}

// bf16 weight copies (both layouts) of every layer from the fp32 master.
void cast_all(rt_net *net, hipStream_t s)
{
    for (int l = 0; l < NL; l++) {
        long o = poff(l);
        nn::launch_cast_weights(taps(l), COUT[l], CIN[l], net->p + o, net->wb + o, net->wt + o, s);
    }
}

// (Re)allocates the activation workspace for grid (nr, nt, np); train adds gradients.
rt_status ensure_ws(rt_net *net, int nr, int nt, int np, bool train)
{
    if (net->nr == nr && net->nt == nt && net->nph == np && (!train || net->train_ws)) return RT_OK;
    if (nr % 4 || nt % 4 || np % 4)
        return nfail(net, RT_EINVAL, "the network needs grid dimensions divisible by 4");
    if ((long)nr * nt * np >= (1L << 31))
        return nfail(net, RT_EINVAL, "the network needs fewer than 2^31 cells");
    free_list(net->ws);
    net->nr = nr; net->nt = nt; net->nph = np;
    net->train_ws = train;
    for (int l = 0; l < 3; l++) {
        Lv &L = net->lv[l];
        L.nr = nr >> l; L.nt = nt >> l; L.np = np >> l;
        L.n = (long)L.nr * L.nt * L.np;
    }
    const long n0 = net->lv[0].n, n1 = net->lv[1].n, n2 = net->lv[2].n;
    auto &W = net->ws;
    net->X = nalloc<bf16>(W, n0 * 16);
    for (int l = 0; l < 10; l++) net->a[l] = nalloc<bf16>(W, net->lv[LEVEL[l]].n * COUT[l]);
    net->p1 = nalloc<bf16>(W, n1 * 16);
    net->p2 = nalloc<bf16>(W, n2 * 32);
    net->z = nalloc<float>(W, n0);
    net->zin = nalloc<float>(W, n0);
    net->lpart = nalloc<double>(W, 2 * 4096);
    net->lres = nalloc<double>(W, 4);
    net->scale = nalloc<double>(W, 2);
    bool ok = net->X && net->p1 && net->p2 && net->z && net->zin && net->lpart && net->lres && net->scale;
    for (int l = 0; l < 10; l++) ok = ok && net->a[l];
    if (train) {
        net->rq = nalloc<float>(W, n0);
        net->gq = nalloc<float>(W, n0);
        ok = ok && net->rq && net->gq;
        net->g9 = nalloc<float>(W, n0 * 16); net->g8 = nalloc<float>(W, n0 * 16);
        net->gU8 = nalloc<float>(W, n0 * 32); net->gS1 = nalloc<float>(W, n0 * 16);
        net->g7 = nalloc<float>(W, n1 * 32); net->g6 = nalloc<float>(W, n1 * 32);
        net->gU6 = nalloc<float>(W, n1 * 64); net->gS2 = nalloc<float>(W, n1 * 32);
        net->g5 = nalloc<float>(W, n2 * 64); net->g4 = nalloc<float>(W, n2 * 64);
        net->gp2 = nalloc<float>(W, n2 * 32); net->g2 = nalloc<float>(W, n1 * 32);
        net->gp1 = nalloc<float>(W, n1 * 16); net->g0 = nalloc<float>(W, n0 * 16);
        net->gz = nalloc<float>(W, n0);
        // partial weight gradients: chunks of 2048 cells x 27 taps x Cout x Cin (max over layers)
        size_t cap = 0;
        for (int l = 0; l < NL - 1; l++)
            cap = std::max(cap, (size_t)nn::wgrad_part_floats(net->lv[LEVEL[l]], COUT[l], CIN[l]));
        cap = std::max(cap, (size_t)((n0 + 2047) / 2048 * 17));
        net->part = nalloc<float>(W, cap);
        net->part_cap = cap;
        ok = ok && net->g9 && net->g8 && net->gU8 && net->gS1 && net->g7 && net->g6 && net->gU6 && net->gS2 &&
             net->g5 && net->g4 && net->gp2 && net->g2 && net->gp1 && net->g0 && net->gz && net->part;
    }
    if (!ok) {
        free_list(net->ws);
        net->nr = net->nt = net->nph = 0;
        return nfail(net, RT_ENOMEM, "network workspace allocation failed");
    }
    return RT_OK;
}

bool conv_fwd(const Lv &L, const bf16 *x1, int c1, int up1, const bf16 *x2, int c2, const bf16 *w, const float *b,
              int cout, int relu, bf16 *y, float *yf, hipStream_t s)
{
    return nn::launch_conv_fwd(L, x1, c1, up1, x2, c2, w, b, cout, relu, y, yf, s);
}

bool conv_bwd_data(const Lv &L, const float *dy, const bf16 *y, int cout, const bf16 *wt, int c1, float *d1, int c2,
                   float *d2, hipStream_t s)
{
    return nn::launch_conv_bwd_data(L, dy, y, cout, wt, c1, d1, c2, d2, s);
}

bool conv_bwd_weight(const Lv &L, const float *dy, const bf16 *y, int cout, const bf16 *x1, int c1, int up1,
                     const bf16 *x2, int c2, float *part, float *dw, float *db, hipStream_t s)
{
    return nn::launch_conv_bwd_weight(L, dy, y, cout, x1, c1, up1, x2, c2, part, dw, db, s);
}

void pool(const Lv &Lc, int C, const bf16 *x, bf16 *y, hipStream_t s) { nn::launch_pool(Lc, C, x, y, s); }

// Forward pass on the workspace input X -> z (fp32, unscaled network output).  With r
// and scale (a preconditioner application): channel 0 of the input is r scale[0], built
// inside the first convolution, and the output scale[1] network(...) goes to zout.
// keep: the last hidden activation is written for a backward pass; otherwise the last
// convolution and the output layer run as one kernel (the same z, bit for bit).
void forward(rt_net *N, hipStream_t s, bool keep, const float *r = nullptr, const double *scale = nullptr,
             float *zout = nullptr)
{
    const Lv *L = N->lv;
    const bf16 *W = N->wb;
    const float *P = N->p;
#define WL(l) (W + poff(l))
#define BL(l) (P + poff(l) + wcount(l))
    if (r) nn::launch_conv_fwd_in(L[0], N->X, r, scale, WL(0), BL(0), N->a[0], s);
    else conv_fwd(L[0], N->X, 16, 0, nullptr, 0, WL(0), BL(0), 16, 1, N->a[0], nullptr, s);
    nn::launch_conv_fwd_pool(L[0], N->a[0], WL(1), BL(1), N->a[1], N->p1, s);  // layer 1 and its pooling
    conv_fwd(L[1], N->p1, 16, 0, nullptr, 0, WL(2), BL(2), 32, 1, N->a[2], nullptr, s);
    conv_fwd(L[1], N->a[2], 32, 0, nullptr, 0, WL(3), BL(3), 32, 1, N->a[3], nullptr, s);
    pool(L[2], 32, N->a[3], N->p2, s);
    conv_fwd(L[2], N->p2, 32, 0, nullptr, 0, WL(4), BL(4), 64, 1, N->a[4], nullptr, s);
    conv_fwd(L[2], N->a[4], 64, 0, nullptr, 0, WL(5), BL(5), 64, 1, N->a[5], nullptr, s);
    conv_fwd(L[1], N->a[5], 64, 1, N->a[3], 32, WL(6), BL(6), 32, 1, N->a[6], nullptr, s);
    conv_fwd(L[1], N->a[6], 32, 0, nullptr, 0, WL(7), BL(7), 32, 1, N->a[7], nullptr, s);
    conv_fwd(L[0], N->a[7], 32, 1, N->a[1], 16, WL(8), BL(8), 16, 1, N->a[8], nullptr, s);
    if (!keep) {
        nn::launch_conv_fwd_head(L[0], N->a[8], WL(9), BL(9), WL(10), BL(10), r ? scale : nullptr, r ? zout : N->z, s);
    } else {
        conv_fwd(L[0], N->a[8], 16, 0, nullptr, 0, WL(9), BL(9), 16, 1, N->a[9], nullptr, s);
        if (r) nn::launch_out_fwd(L[0].n, N->a[9], WL(10), BL(10), scale, zout, s);
        else nn::launch_out_fwd(L[0].n, N->a[9], WL(10), BL(10), nullptr, N->z, s);
    }
}

// Backward pass for dL/dz = N->gz: parameter gradients into N->g.
void backward(rt_net *N, hipStream_t s)
{
    const Lv *L = N->lv;
    const bf16 *WT = N->wt, *W = N->wb;
    float *G = N->g;
#define GW(l) (G + poff(l))
#define GB(l) (G + poff(l) + wcount(l))
#define WTL(l) (WT + poff(l))
    const long n0 = L[0].n;
    nn::launch_out_bwd(n0, N->a[9], W + poff(10), N->gz, N->g9, N->part, GW(10), s);  // 1x1 output layer
    conv_bwd_weight(L[0], N->g9, N->a[9], 16, N->a[8], 16, 0, nullptr, 0, N->part, GW(9), GB(9), s);
    conv_bwd_data(L[0], N->g9, N->a[9], 16, WTL(9), 16, N->g8, 0, nullptr, s);
    conv_bwd_weight(L[0], N->g8, N->a[8], 16, N->a[7], 32, 1, N->a[1], 16, N->part, GW(8), GB(8), s);
    conv_bwd_data(L[0], N->g8, N->a[8], 16, WTL(8), 32, N->gU8, 16, N->gS1, s);
    nn::launch_up_bwd(L[1], 32, N->gU8, N->g7, s);
    conv_bwd_weight(L[1], N->g7, N->a[7], 32, N->a[6], 32, 0, nullptr, 0, N->part, GW(7), GB(7), s);
    conv_bwd_data(L[1], N->g7, N->a[7], 32, WTL(7), 32, N->g6, 0, nullptr, s);
    conv_bwd_weight(L[1], N->g6, N->a[6], 32, N->a[5], 64, 1, N->a[3], 32, N->part, GW(6), GB(6), s);
    conv_bwd_data(L[1], N->g6, N->a[6], 32, WTL(6), 64, N->gU6, 32, N->gS2, s);
    nn::launch_up_bwd(L[2], 64, N->gU6, N->g5, s);
    conv_bwd_weight(L[2], N->g5, N->a[5], 64, N->a[4], 64, 0, nullptr, 0, N->part, GW(5), GB(5), s);
    conv_bwd_data(L[2], N->g5, N->a[5], 64, WTL(5), 64, N->g4, 0, nullptr, s);
    conv_bwd_weight(L[2], N->g4, N->a[4], 64, N->p2, 32, 0, nullptr, 0, N->part, GW(4), GB(4), s);
    conv_bwd_data(L[2], N->g4, N->a[4], 64, WTL(4), 32, N->gp2, 0, nullptr, s);
    nn::launch_pool_bwd_add(L[1], 32, N->gp2, N->gS2, s);
    conv_bwd_weight(L[1], N->gS2, N->a[3], 32, N->a[2], 32, 0, nullptr, 0, N->part, GW(3), GB(3), s);
    conv_bwd_data(L[1], N->gS2, N->a[3], 32, WTL(3), 32, N->g2, 0, nullptr, s);
    conv_bwd_weight(L[1], N->g2, N->a[2], 32, N->p1, 16, 0, nullptr, 0, N->part, GW(2), GB(2), s);
    conv_bwd_data(L[1], N->g2, N->a[2], 32, WTL(2), 16, N->gp1, 0, nullptr, s);
    nn::launch_pool_bwd_add(L[0], 16, N->gp1, N->gS1, s);
    conv_bwd_weight(L[0], N->gS1, N->a[1], 16, N->a[0], 16, 0, nullptr, 0, N->part, GW(1), GB(1), s);
    conv_bwd_data(L[0], N->gS1, N->a[1], 16, WTL(1), 16, N->g0, 0, nullptr, s);
    conv_bwd_weight(L[0], N->g0, N->a[0], 16, N->X, 16, 0, nullptr, 0, N->part, GW(0), GB(0), s);
}

void loss(rt_net *N, const float *e, hipStream_t s)
{
    nn::launch_loss(N->lv[0].n, N->z, e, N->lpart, N->lres, N->gz, s);
}

// He-style initialisation from a counter-based hash of (seed, index): uniform in
// [-sqrt(6/fan_in), sqrt(6/fan_in)] for weights, zero biases.
void init_params(std::vector<float> &h, unsigned seed)
{
    h.assign(poff(NL), 0.0f);
    for (int l = 0; l < NL; l++) {
        long o = poff(l);
        double bound = std::sqrt(6.0 / (taps(l) * CIN[l]));
        if (l == NL - 1) bound *= 0.1;
        for (long i = 0; i < wcount(l); i++) {
            uint64_t x = ((uint64_t)seed << 32) ^ (uint64_t)(o + i) * 0x9E3779B97F4A7C15ull;
            x ^= x >> 30; x *= 0xBF58476D1CE4E5B9ull; x ^= x >> 27; x *= 0x94D049BB133111EBull; x ^= x >> 31;
            double u = (double)(x >> 11) * (1.0 / 9007199254740992.0);
            h[o + i] = (float)((2.0 * u - 1.0) * bound);
        }
    }
}

}  // namespace

// ===================================================================== C-ABI

extern "C" {

rt_status rt_net_create(const rt_net_config *cfg, rt_net **out)
{
    if (!out) return nfail(nullptr, RT_EINVAL, "rt_net_create: out is NULL");
    *out = nullptr;
    rt_net *net = new (std::nothrow) rt_net();
    if (!net) return nfail(nullptr, RT_ENOMEM, "out of host memory");
    (void)hipGetDevice(&net->device);
    net->np_ = poff(NL);
    net->p = nalloc<float>(net->allocs, net->np_);
    net->g = nalloc<float>(net->allocs, net->np_);
    net->m = nalloc<float>(net->allocs, net->np_);
    net->v = nalloc<float>(net->allocs, net->np_);
    net->wb = nalloc<bf16>(net->allocs, net->np_);
    net->wt = nalloc<bf16>(net->allocs, net->np_);
    if (!net->p || !net->g || !net->m || !net->v || !net->wb || !net->wt) {
        rt_net_destroy(net);
        return nfail(nullptr, RT_ENOMEM, "rt_net_create: out of device memory");
    }
    std::vector<float> h;
    init_params(h, cfg ? cfg->seed : 1u);
    if (hipMemcpy(net->p, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(net->m, 0, h.size() * sizeof(float)) != hipSuccess ||
        hipMemset(net->v, 0, h.size() * sizeof(float)) != hipSuccess ||
        hipMemset(net->g, 0, h.size() * sizeof(float)) != hipSuccess) {
        rt_net_destroy(net);
        return nfail(nullptr, RT_EDEVICE, "rt_net_create: upload failed");
    }
    cast_all(net, nullptr);
    if (hipDeviceSynchronize() != hipSuccess) {
        rt_net_destroy(net);
        return nfail(nullptr, RT_EDEVICE, "rt_net_create: cast failed");
    }
    *out = net;
    return RT_OK;
}

void rt_net_destroy(rt_net *net)
{
    if (!net) return;
    (void)hipDeviceSynchronize();
    free_list(net->ws);
    free_list(net->allocs);
    delete net;
}

const char *rt_net_last_error(const rt_net *net) { return net ? net->err.c_str() : g_nerr.c_str(); }

long rt_net_param_count(const rt_net *net) { return net ? net->np_ : poff(NL); }

rt_status rt_net_get_params(const rt_net *net, float *host, long n)
{
    if (!net || !host || n != net->np_) return nfail(const_cast<rt_net *>(net), RT_EINVAL, "rt_net_get_params: bad args");
    NN_HIP(const_cast<rt_net *>(net), hipDeviceSynchronize());
    NN_HIP(const_cast<rt_net *>(net), hipMemcpy(host, net->p, n * sizeof(float), hipMemcpyDeviceToHost));
    return RT_OK;
}

rt_status rt_net_get_grads(const rt_net *net, float *host, long n)
{
    if (!net || !host || n != net->np_) return nfail(const_cast<rt_net *>(net), RT_EINVAL, "rt_net_get_grads: bad args");
    NN_HIP(const_cast<rt_net *>(net), hipDeviceSynchronize());
    NN_HIP(const_cast<rt_net *>(net), hipMemcpy(host, net->g, n * sizeof(float), hipMemcpyDeviceToHost));
    return RT_OK;
}

rt_status rt_net_set_params(rt_net *net, const float *host, long n)
{
    if (!net || !host || n != net->np_) return nfail(net, RT_EINVAL, "rt_net_set_params: bad args");
    for (long i = 0; i < n; i++)
        if (!std::isfinite(host[i])) return nfail(net, RT_ENONFINITE, "rt_net_set_params: non-finite parameter");
    NN_HIP(net, hipDeviceSynchronize());
    NN_HIP(net, hipMemcpy(net->p, host, n * sizeof(float), hipMemcpyHostToDevice));
    NN_HIP(net, hipMemset(net->m, 0, n * sizeof(float)));
    NN_HIP(net, hipMemset(net->v, 0, n * sizeof(float)));
    net->adam_t = 0;
    cast_all(net, nullptr);
    NN_HIP(net, hipDeviceSynchronize());
    return RT_OK;
}

rt_status rt_net_forward(rt_ctx *ctx, rt_net *net, const void *X, float *z)
{
    if (!ctx || !net || !X || !z) return nfail(net, RT_EINVAL, "rt_net_forward: NULL argument");
    if (rt_status e = ensure_ws(net, ctx->d.nr, ctx->d.nt, ctx->d.np, false)) return e;
    hipStream_t s = ctx->stream;
    NN_HIP(net, hipMemcpyAsync(net->X, X, net->lv[0].n * 16 * sizeof(bf16), hipMemcpyDeviceToDevice, s));
    forward(net, s, false);
    NN_HIP(net, hipMemcpyAsync(z, net->z, net->lv[0].n * sizeof(float), hipMemcpyDeviceToDevice, s));
    NN_HIP(net, hipGetLastError());
    return RT_OK;
}

rt_status rt_net_apply(rt_ctx *ctx, rt_net *net, const float *r, float *z)
{
    if (!ctx || !net || !r || !z) return nfail(net, RT_EINVAL, "rt_net_apply: NULL argument");
    if (!ctx->have_system) return nfail(net, RT_EINVAL, "rt_net_apply: no assembled system on the context");
    if (rt_status e = net_prepare(net, ctx)) return e;
    launch_norm2_rr32(ctx->d, ctx->nblk, r, ctx->partials, ctx->counter, ctx->sc, ctx->stream);
    return net_precond(net, ctx, r, z);
}

rt_status rt_net_loss_grad(rt_ctx *ctx, rt_net *net, const void *X, const float *e, float *z, double *loss_out)
{
    if (!ctx || !net || !X || !e) return nfail(net, RT_EINVAL, "rt_net_loss_grad: NULL argument");
    if (rt_status er = ensure_ws(net, ctx->d.nr, ctx->d.nt, ctx->d.np, true)) return er;
    hipStream_t s = ctx->stream;
    NN_HIP(net, hipMemcpyAsync(net->X, X, net->lv[0].n * 16 * sizeof(bf16), hipMemcpyDeviceToDevice, s));
    forward(net, s, true);
    loss(net, e, s);
    backward(net, s);
    if (z) NN_HIP(net, hipMemcpyAsync(z, net->z, net->lv[0].n * sizeof(float), hipMemcpyDeviceToDevice, s));
    NN_HIP(net, hipGetLastError());
    if (loss_out) {
        double h[2];
        NN_HIP(net, hipMemcpyAsync(h, net->lres, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        NN_HIP(net, hipStreamSynchronize(s));
        *loss_out = h[0];
    }
    return RT_OK;
}

rt_status rt_net_loss_grad_resid(rt_ctx *ctx, rt_net *net, const void *X, const float *r, const float *a32, float *z,
                                 double *loss_out)
{
    if (!ctx || !net || !X || !r || !a32) return nfail(net, RT_EINVAL, "rt_net_loss_grad_resid: NULL argument");
    if (rt_status er = ensure_ws(net, ctx->d.nr, ctx->d.nt, ctx->d.np, true)) return er;
    hipStream_t s = ctx->stream;
    const long n = net->lv[0].n;
    NN_HIP(net, hipMemcpyAsync(net->X, X, n * 16 * sizeof(bf16), hipMemcpyDeviceToDevice, s));
    forward(net, s, true);
    launch_spmv32(ctx->d, ctx->nblk, a32, net->z, net->rq, s);                    // A z
    nn::launch_loss(n, net->rq, r, net->lpart, net->lres, net->gq, s);           // L, dL/d(A z)
    launch_spmv32(ctx->d, ctx->nblk, a32, net->gq, net->gz, s);                   // dL/dz = A^T dL/d(A z)
    backward(net, s);
    if (z) NN_HIP(net, hipMemcpyAsync(z, net->z, n * sizeof(float), hipMemcpyDeviceToDevice, s));
    NN_HIP(net, hipGetLastError());
    if (loss_out) {
        double h[2];
        NN_HIP(net, hipMemcpyAsync(h, net->lres, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        NN_HIP(net, hipStreamSynchronize(s));
        *loss_out = h[0];
    }
    return RT_OK;
}

rt_status rt_net_adam(rt_ctx *ctx, rt_net *net, double lr)
{
    if (!ctx || !net || !(lr > 0.0)) return nfail(net, RT_EINVAL, "rt_net_adam: bad arguments");
    hipStream_t s = ctx->stream;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    net->adam_t++;
    float c1 = 1.0f - std::pow(b1, (float)net->adam_t), c2 = 1.0f - std::pow(b2, (float)net->adam_t);
    nn::launch_adam(net->np_, net->p, net->g, net->m, net->v, (float)lr, b1, b2, eps, c1, c2, s);
    cast_all(net, s);
    NN_HIP(net, hipGetLastError());
    return RT_OK;
}

rt_status rt_net_save(const rt_net *net, const char *path)
{
    if (!net || !path) return nfail(const_cast<rt_net *>(net), RT_EINVAL, "rt_net_save: bad arguments");
    std::vector<float> h(net->np_);
    if (rt_status e = rt_net_get_params(net, h.data(), net->np_)) return e;
    FILE *f = std::fopen(path, "wb");
    if (!f) return nfail(const_cast<rt_net *>(net), RT_EINVAL, std::string("cannot open ") + path);
    const char magic[8] = {'R', 'T', 'M', 'I', 'N', 'E', 'T', '1'};
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(&net->np_, sizeof(long), 1, f) == 1 &&
              std::fwrite(h.data(), sizeof(float), h.size(), f) == h.size();
    std::fclose(f);
    return ok ? RT_OK : nfail(const_cast<rt_net *>(net), RT_EINVAL, "rt_net_save: write failed");
}

rt_status rt_net_load(rt_net *net, const char *path)
{
    if (!net || !path) return nfail(net, RT_EINVAL, "rt_net_load: bad arguments");
    FILE *f = std::fopen(path, "rb");
    if (!f) return nfail(net, RT_EINVAL, std::string("cannot open ") + path);
    char magic[8];
    long n = 0;
    std::vector<float> h(net->np_);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "RTMINET1", 8) == 0 &&
              std::fread(&n, sizeof(long), 1, f) == 1 && n == net->np_ &&
              std::fread(h.data(), sizeof(float), h.size(), f) == h.size();
    std::fclose(f);
    if (!ok) return nfail(net, RT_EINVAL, "rt_net_load: not a network file of this architecture");
    return rt_net_set_params(net, h.data(), net->np_);
}

// ------------------------------------------------------------ layer-level calls

rt_status rt_nn_conv3d_fwd(void *stream, int nr, int nt, int np, const void *x1, int c1, int up1, const void *x2,
                           int c2, const void *w, const float *bias, int cout, int relu, void *y, float *yf)
{
    if (nr < 1 || nt < 1 || np < 1 || !x1 || c1 % 16 || c2 % 16 || c1 < 16 || (c2 && !x2) || !w || cout % 16 ||
        cout < 16 || cout > 64 || (!y && !yf) || (up1 && (nr % 2 || nt % 2 || np % 2)) ||
        (long)nr * nt * np >= (1L << 31))
        return nfail(nullptr, RT_EINVAL, "rt_nn_conv3d_fwd: bad arguments");
    Lv L{nr, nt, np, (long)nr * nt * np};
    conv_fwd(L, (const bf16 *)x1, c1, up1, (const bf16 *)x2, c2, (const bf16 *)w, bias, cout, relu, (bf16 *)y, yf,
             (hipStream_t)stream);
    NN_HIP(nullptr, hipGetLastError());
    return RT_OK;
}

rt_status rt_nn_conv3d_fwd_pool(void *stream, int nr, int nt, int np, const void *x, const void *w, const float *bias,
                                void *y, void *yp)
{
    if (nr < 2 || nt < 2 || np < 2 || nr % 2 || nt % 2 || np % 2 || !x || !w || !bias || !y || !yp ||
        (long)nr * nt * np >= (1L << 31))
        return nfail(nullptr, RT_EINVAL, "rt_nn_conv3d_fwd_pool: bad arguments");
    Lv L{nr, nt, np, (long)nr * nt * np};
    nn::launch_conv_fwd_pool(L, (const bf16 *)x, (const bf16 *)w, bias, (bf16 *)y, (bf16 *)yp, (hipStream_t)stream);
    NN_HIP(nullptr, hipGetLastError());
    return RT_OK;
}

rt_status rt_nn_conv3d_bwd_data(void *stream, int nr, int nt, int np, const float *dy, const void *yrelu, int cout,
                                const void *wt, int c1, float *d1, int c2, float *d2)
{
    if (nr < 1 || nt < 1 || np < 1 || !dy || cout % 16 || cout < 16 || !wt || c1 % 16 || c2 % 16 || c1 < 16 || !d1 ||
        (c2 && !d2) || ((c1 + c2) / 16 == 5) || (c1 + c2) > 96 || (long)nr * nt * np >= (1L << 31))
        return nfail(nullptr, RT_EINVAL, "rt_nn_conv3d_bwd_data: bad arguments");
    Lv L{nr, nt, np, (long)nr * nt * np};
    conv_bwd_data(L, dy, (const bf16 *)yrelu, cout, (const bf16 *)wt, c1, d1, c2, d2, (hipStream_t)stream);
    NN_HIP(nullptr, hipGetLastError());
    return RT_OK;
}

rt_status rt_nn_conv3d_bwd_weight(void *stream, int nr, int nt, int np, const float *dy, const void *yrelu, int cout,
                                  const void *x1, int c1, int up1, const void *x2, int c2, float *dw, float *db)
{
    if (nr < 1 || nt < 1 || np < 1 || !dy || cout % 16 || cout < 16 || cout > 64 || !x1 || c1 % 16 || c2 % 16 ||
        c1 < 16 || (c2 && !x2) || !dw || !db || (up1 && (nr % 2 || nt % 2 || np % 2)))
        return nfail(nullptr, RT_EINVAL, "rt_nn_conv3d_bwd_weight: bad arguments");
    Lv L{nr, nt, np, (long)nr * nt * np};
    float *part = nullptr;
    const size_t cap = (size_t)nn::wgrad_part_floats(L, cout, c1 + c2);
    NN_HIP(nullptr, hipMalloc(&part, cap * sizeof(float)));
    if (!conv_bwd_weight(L, dy, (const bf16 *)yrelu, cout, (const bf16 *)x1, c1, up1, (const bf16 *)x2, c2, part, dw,
                         db, (hipStream_t)stream)) {
        (void)hipFree(part);
        return nfail(nullptr, RT_EINVAL, "rt_nn_conv3d_bwd_weight: unsupported channel counts");
    }
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    (void)hipFree(part);
    if (e != hipSuccess) return nfail(nullptr, RT_EDEVICE, hipGetErrorString(e));
    return RT_OK;
}

// Scratch of rt_nn_conv3d_bwd_weight_noalloc: the per-block partial sums of the weight
// gradient, then of the bias gradient (every float the kernels read is written first in
// the same call, so nothing needs clearing).  Each device holds its own copy until the
// process ends; host code uses the device address from hipGetSymbolAddress, never the
// array's name.
constexpr long kWgradScratchFloats = 8L << 20;  // 32 MiB
static __device__ __align__(256) float scratch[kWgradScratchFloats];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch[kMaxDevices] = {};

// The current device's address of `scratch`, looked up once per device.
rt_status scratch_ptr(float **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return nfail(nullptr, RT_EDEVICE, "rt_nn_conv3d_bwd_weight_noalloc: no usable current device");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return nfail(nullptr, RT_EDEVICE, std::string("rt_nn_conv3d_bwd_weight_noalloc: hipGetSymbolAddress: ") +
                                                  hipGetErrorString(e));
        g_scratch[dev] = static_cast<float *>(p);
    }
    *out = g_scratch[dev];
    return RT_OK;
}
}  // namespace

rt_status rt_nn_conv3d_bwd_weight_noalloc(void *stream, int nr, int nt, int np, const float *dy, const void *yrelu,
                                          int cout, const void *x1, int c1, int up1, const void *x2, int c2, float *dw,
                                          float *db)
{
    if (nr < 1 || nt < 1 || np < 1 || !dy || cout % 16 || cout < 16 || cout > 64 || !x1 || c1 % 16 || c2 % 16 ||
        c1 < 16 || (c2 && !x2) || !dw || !db || (up1 && (nr % 2 || nt % 2 || np % 2)))
        return nfail(nullptr, RT_EINVAL, "rt_nn_conv3d_bwd_weight_noalloc: bad arguments");
    Lv L{nr, nt, np, (long)nr * nt * np};
    const long need = nn::wgrad_part_floats(L, cout, c1 + c2);
    if (need > kWgradScratchFloats)
        return nfail(nullptr, RT_EINVAL,
                     "rt_nn_conv3d_bwd_weight_noalloc: the layer needs " + std::to_string(need) +
                         " floats of partial sums, more than the " + std::to_string(kWgradScratchFloats) +
                         " of the static scratch (use rt_nn_conv3d_bwd_weight)");
    float *part = nullptr;
    if (rt_status e = scratch_ptr(&part)) return e;
    if (!conv_bwd_weight(L, dy, (const bf16 *)yrelu, cout, (const bf16 *)x1, c1, up1, (const bf16 *)x2, c2, part, dw,
                         db, (hipStream_t)stream))
        return nfail(nullptr, RT_EINVAL, "rt_nn_conv3d_bwd_weight_noalloc: unsupported channel counts");
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return nfail(nullptr, RT_EDEVICE, hipGetErrorString(e));
    return RT_OK;
}

// --------------------------------------------------------------- training set

rt_status rt_dataset_create(rt_ctx *ctx, int capacity, rt_dataset **out)
{
    if (!ctx || !out || capacity < 1) return nfail(nullptr, RT_EINVAL, "rt_dataset_create: bad arguments");
    rt_dataset *ds = new (std::nothrow) rt_dataset();
    if (!ds) return nfail(nullptr, RT_ENOMEM, "out of host memory");
    ds->n = ctx->d.n;
    ds->cap = capacity;
    ds->nr = ctx->d.nr; ds->nt = ctx->d.nt; ds->nph = ctx->d.np;
    ds->X = nalloc<bf16>(ds->allocs, (size_t)capacity * ds->n * 16);
    ds->E = nalloc<float>(ds->allocs, (size_t)capacity * ds->n);
    ds->R = nalloc<float>(ds->allocs, (size_t)capacity * ds->n);
    ds->A32 = nalloc<float>(ds->allocs, (size_t)capacity * 3 * ds->n);
    ds->ystar = nalloc<double>(ds->allocs, ds->n);
    ds->y0 = nalloc<double>(ds->allocs, ds->n);
    if (!ds->X || !ds->E || !ds->R || !ds->A32 || !ds->ystar || !ds->y0) {
        rt_dataset_destroy(ds);
        return nfail(nullptr, RT_ENOMEM, "rt_dataset_create: out of device memory");
    }
    *out = ds;
    return RT_OK;
}

void rt_dataset_destroy(rt_dataset *ds)
{
    if (!ds) return;
    (void)hipDeviceSynchronize();
    free_list(ds->allocs);
    delete ds;
}

int rt_dataset_size(const rt_dataset *ds) { return ds ? ds->size : 0; }

}  // extern "C"

namespace {

// Pairs from k iterations of the float64 CG (net == nullptr) or of the learned flexible
// CG with the network net, for each k in iters, all from E0.
rt_status add_pairs(rt_ctx *ctx, rt_dataset *ds, rt_net *net, const double *E0, const int *iters, int n_iters)
{
    if (!ctx || !ds || !E0 || !iters || n_iters < 1) return nfail(nullptr, RT_EINVAL, "rt_dataset_add: bad arguments");
    if (ctx->d.nr != ds->nr || ctx->d.nt != ds->nt || ctx->d.np != ds->nph)
        return nfail(nullptr, RT_EINVAL, "rt_dataset_add: context grid differs from the set's");
    if (ds->size + n_iters > ds->cap) return nfail(nullptr, RT_EINVAL, "rt_dataset_add: set is full");
    if (!ctx->have_system) return nfail(nullptr, RT_EINVAL, "rt_dataset_add: no assembled system");
    for (int q = 0; q < n_iters; q++)
        if (iters[q] < 0) return nfail(nullptr, RT_EINVAL, "rt_dataset_add: negative iteration count");
    hipStream_t s = ctx->stream;
    const long n = ds->n;
    // start y0 = E0 / s and the reference y* (float64 CG to 1e-12)
    launch_scale_div(n, ctx->s, E0, ds->y0, s);
    NN_HIP(nullptr, hipMemcpyAsync(ds->ystar, ds->y0, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (rt_status e = solve_fp64_from(ctx, 1e-12, 200000, ds->ystar, nullptr))
        return nfail(nullptr, e, std::string("reference solve: ") + rt_last_error(ctx));
    const int fld = ds->nfield;
    NN_HIP(nullptr, hipMemcpyAsync(ds->A32 + (size_t)fld * 3 * n, ctx->ahat32, 3 * n * sizeof(float),
                                   hipMemcpyDeviceToDevice, s));
    double *y = ctx->qv;  // scratch: the Krylov q vector is free between solves
    for (int q = 0; q < n_iters; q++) {
        NN_HIP(nullptr, hipMemcpyAsync(y, ds->y0, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (iters[q] > 0) {
            rt_status e = net ? learned_from(ctx, net, iters[q], y, nullptr)
                              : solve_fp64_from(ctx, 1e-30, iters[q], y, nullptr);
            if (e) return nfail(nullptr, e, std::string("partial solve: ") + rt_last_error(ctx));
        }
        launch_resid(ctx->d, ctx->nblk, ctx->ahat, ctx->bhat, y, ctx->r, ctx->partials, ctx->counter, ctx->sc, 0, s);
        bf16 *X = ds->X + (size_t)ds->size * n * 16;
        float *E = ds->E + (size_t)ds->size * n;
        nn::launch_pair(n, ctx->sc, ds->ystar, y, ctx->nscale, E, s);
        nn::launch_features(n, ctx->ahat, X, s);
        nn::launch_set_input(n, (const double *)ctx->r, ctx->nscale, X, s);
        nn::launch_scaled_f32(n, ctx->r, ctx->nscale, ds->R + (size_t)ds->size * n, s);
        NN_HIP(nullptr, hipGetLastError());
        ds->field.push_back(fld);
        ds->size++;
    }
    ds->nfield++;
    NN_HIP(nullptr, hipStreamSynchronize(s));
    return RT_OK;
}

}  // namespace

extern "C" {

rt_status rt_dataset_add(rt_ctx *ctx, rt_dataset *ds, const double *E0, const int *iters, int n_iters)
{
    return add_pairs(ctx, ds, nullptr, E0, iters, n_iters);
}

rt_status rt_dataset_add_learned(rt_ctx *ctx, rt_dataset *ds, rt_net *net, const double *E0, const int *iters,
                                 int n_iters)
{
    if (!net) return nfail(nullptr, RT_EINVAL, "rt_dataset_add_learned: network is NULL");
    return add_pairs(ctx, ds, net, E0, iters, n_iters);
}

rt_status rt_net_train(rt_ctx *ctx, rt_net *net, rt_dataset *ds, const rt_train_opts *o, rt_train_stats *st)
{
    if (!ctx || !net || !ds || !o || o->epochs < 1 || !(o->lr > 0.0) ||
        (o->loss != RT_LOSS_ERROR && o->loss != RT_LOSS_RESIDUAL))
        return nfail(net, RT_EINVAL, "rt_net_train: bad arguments");
    if (ds->size < 1) return nfail(net, RT_EINVAL, "rt_net_train: empty set");
    if (ctx->d.nr != ds->nr || ctx->d.nt != ds->nt || ctx->d.np != ds->nph)
        return nfail(net, RT_EINVAL, "rt_net_train: context grid differs from the set's");
    auto t0 = std::chrono::steady_clock::now();
    const long n = ds->n;
    std::vector<int> order(ds->size);
    rt_train_stats S{};
    const int total = o->epochs * ds->size;
    int step = 0;
    for (int ep = 0; ep < o->epochs; ep++) {
        for (int q = 0; q < ds->size; q++) order[q] = q;
        uint64_t x = 0x9E3779B97F4A7C15ull * (uint64_t)(o->seed + 1) + (uint64_t)ep;
        for (int q = ds->size - 1; q > 0; q--) {  // Fisher-Yates with a splitmix64 stream
            x += 0x9E3779B97F4A7C15ull;
            uint64_t zz = x;
            zz = (zz ^ (zz >> 30)) * 0xBF58476D1CE4E5B9ull;
            zz = (zz ^ (zz >> 27)) * 0x94D049BB133111EBull;
            zz ^= zz >> 31;
            int j = (int)(zz % (uint64_t)(q + 1));
            std::swap(order[q], order[j]);
        }
        double sum = 0.0;
        for (int q = 0; q < ds->size; q++, step++) {
            const int idx = order[q];
            double L = 0.0;
            const bf16 *Xi = ds->X + (size_t)idx * n * 16;
            rt_status e = (o->loss == RT_LOSS_RESIDUAL)
                              ? rt_net_loss_grad_resid(ctx, net, Xi, ds->R + (size_t)idx * n,
                                                       ds->A32 + (size_t)ds->field[idx] * 3 * n, nullptr, &L)
                              : rt_net_loss_grad(ctx, net, Xi, ds->E + (size_t)idx * n, nullptr, &L);
            if (e) return e;
            if (!std::isfinite(L)) return nfail(net, RT_ENONFINITE, "rt_net_train: loss is not finite");
            sum += L;
            const double frac = total > 1 ? (double)step / (total - 1) : 0.0;
            const double lr = o->lr * (0.1 + 0.9 * 0.5 * (1.0 + std::cos(M_PI * frac)));
            if (rt_status e = rt_net_adam(ctx, net, lr)) return e;
        }
        const double mean = sum / ds->size;
        if (ep == 0) S.loss_first_epoch = mean;
        S.loss_last_epoch = mean;
    }
    NN_HIP(net, hipStreamSynchronize(ctx->stream));
    S.steps = step;
    S.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (st) *st = S;
    return RT_OK;
}

}  // extern "C"

namespace rt {

rt_status net_prepare(rt_net *net, rt_ctx *ctx)
{
    if (rt_status e = ensure_ws(net, ctx->d.nr, ctx->d.nt, ctx->d.np, net->train_ws)) return e;
    nn::launch_features(ctx->d.n, ctx->ahat, net->X, ctx->stream);
    NN_HIP(net, hipGetLastError());
    return RT_OK;
}

rt_status net_precond(rt_net *net, rt_ctx *ctx, const float *r, float *z)
{
    hipStream_t s = ctx->stream;
    const long n = ctx->d.n;
    launch_rms_scale(n, ctx->sc, ctx->nscale, s);
    forward(net, s, false, r, ctx->nscale, z);
    NN_HIP(net, hipGetLastError());
    return RT_OK;
}

}  // namespace rt
