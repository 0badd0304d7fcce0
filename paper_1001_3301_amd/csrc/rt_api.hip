// Host side of the librtmi C-ABI: argument checks, context and workspaces, the
// problem tables, Eq. (20) bin fluxes, and the solver drivers that sequence the
// kernels of the radiation step (Fig. 1 of Kuiper et al.).
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <new>

#include "rt_internal.h"

using namespace rt;

namespace rt {
void raytrace_prepare();
}

namespace {

thread_local std::string g_err;  // errors of rt_create (no context yet)

rt_status fail(rt_ctx *ctx, rt_status s, const std::string &m)
{
    if (ctx) ctx->err = m; else g_err = m;
    return s;
}

#define RT_HIP(ctx, call)                                                                         \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail((ctx), RT_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

#define RT_CHECK(ctx, cond, msg)                                                                  \
    do {                                                                                          \
        if (!(cond)) return fail((ctx), RT_EINVAL, (msg));                                        \
    } while (0)

template <class T>
T *dalloc(rt_ctx *ctx, size_t n)
{
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return nullptr;
    ctx->allocs.push_back(p);
    return static_cast<T *>(p);
}

bool isfin(double x) { return std::isfinite(x); }

// log-log interpolation of a mean-opacity column on the host (used once per system
// for kappa_R at the boundary temperature).
double host_mean(const std::vector<double> &T, const std::vector<double> &tab, double t)
{
    size_t n = T.size();
    if (t <= T[0]) return tab[0];
    if (t >= T[n - 1]) return tab[n - 1];
    size_t k = 0;
    while (T[k + 1] <= t) k++;
    double l0 = std::log(T[k]), l1 = std::log(T[k + 1]);
    double lw = (std::log(t) - l0) / (l1 - l0);
    return std::exp((1.0 - lw) * std::log(tab[k]) + lw * std::log(tab[k + 1]));
}

rt_status read_scalars(rt_ctx *ctx)
{
    RT_HIP(ctx, hipMemcpyAsync(ctx->h_sc, ctx->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, ctx->stream));
    RT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return RT_OK;
}

rt_status write_scalars(rt_ctx *ctx)
{
    RT_HIP(ctx, hipMemcpyAsync(ctx->sc, ctx->h_sc, sizeof(DevScalars), hipMemcpyHostToDevice, ctx->stream));
    RT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return RT_OK;
}

rt_status check_fld(rt_ctx *ctx, const rt_fld_params *p)
{
    RT_CHECK(ctx, p, "rt_fld_params is NULL");
    RT_CHECK(ctx, p->dt > 0.0 && isfin(p->dt), "dt must be positive");
    RT_CHECK(ctx, p->c_V >= 0.0 && isfin(p->c_V), "c_V must be >= 0");
    RT_CHECK(ctx, p->T_bc > 0.0 && isfin(p->T_bc), "T_bc must be positive");
    RT_CHECK(ctx, p->E_floor >= 0.0 && isfin(p->E_floor), "E_floor must be >= 0");
    return RT_OK;
}

// ---------------------------------------------------------------- Eq. (20)

// Planck integrals in x = h nu / (k T):
//   P(x) = int_0^x t^3/(e^t - 1) dt = sum_n c_n x^{n+3}/(n+3) for x <= 1, with
//          t/(e^t - 1) = sum_n c_n t^n (c_n = B_n / n!: c_0 = 1, sum_{k<=n} c_k/(n+1-k)! = 0);
//   Q(x) = int_x^inf = sum_m e^{-m x}(x^3/m + 3x^2/m^2 + 6x/m^3 + 6/m^4) for x > 1;
// each extended to the other side with P + Q = pi^4/15.
const double kPi4_15 = 6.4939394022668291491;  // pi^4 / 15

double planck_P_series(double x)
{
    static double c[48];
    static bool init = false;
    if (!init) {
        double fact[50];
        fact[0] = 1.0;
        for (int i = 1; i < 50; i++) fact[i] = fact[i - 1] * i;
        c[0] = 1.0;
        for (int n = 1; n < 48; n++) {
            double s = 0.0;
            for (int k = 0; k < n; k++) s += c[k] / fact[n + 1 - k];
            c[n] = -s;
        }
        init = true;
    }
    double P = 0.0, xp = x * x * x;
    for (int n = 0; n < 48; n++) {
        P += c[n] * xp / (n + 3);
        xp *= x;
    }
    return P;
}

double planck_Q_series(double x)
{
    double s = 0.0;
    for (int m = 1; m < 400; m++) {
        double e = std::exp(-m * x);
        double t = e * (x * x * x / m + 3.0 * x * x / ((double)m * m) + 6.0 * x / ((double)m * m * m) +
                        6.0 / ((double)m * m * m * m));
        s += t;
        if (t < 1e-19 * s) break;
    }
    return s;
}

double planck_P(double x) { return x <= 0.0 ? 0.0 : (x <= 1.0 ? planck_P_series(x) : kPi4_15 - planck_Q_series(x)); }
double planck_Q(double x) { return x <= 1.0 ? kPi4_15 - planck_P(x) : planck_Q_series(x); }

// int_lo^hi t^3/(e^t - 1) dt without cancellation: below x = 1 from P, above from Q.
double planck_band(double lo, double hi)
{
    if (hi <= 1.0) return planck_P(hi) - planck_P(lo);
    if (lo >= 1.0) return planck_Q(lo) - (std::isinf(hi) ? 0.0 : planck_Q(hi));
    return (planck_P(1.0) - planck_P(lo)) + (planck_Q(1.0) - (std::isinf(hi) ? 0.0 : planck_Q(hi)));
}

}  // namespace

// ==================================================================== C-ABI

extern "C" {

const char *rt_last_error(const rt_ctx *ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

long rt_ncell(const rt_ctx *ctx) { return ctx ? ctx->d.n : 0; }

rt_status rt_star_bin_flux(double T_star, int n_nu, const double *nu, double *F_out)
{
    if (!(T_star > 0.0) || n_nu < 1 || !nu || !F_out) return fail(nullptr, RT_EINVAL, "rt_star_bin_flux: bad arguments");
    for (int i = 1; i < n_nu; i++)
        if (!(nu[i] > nu[i - 1])) return fail(nullptr, RT_EINVAL, "rt_star_bin_flux: nu must increase");
    if (!(nu[0] > 0.0)) return fail(nullptr, RT_EINVAL, "rt_star_bin_flux: nu must be positive");
    const double xs = kH / (kBoltz * T_star);
    const double norm = kSigma * std::pow(T_star, 4) * 15.0 / std::pow(M_PI, 4);
    for (int i = 0; i < n_nu; i++) {
        double lo = (i == 0) ? 0.0 : 0.5 * (nu[i - 1] + nu[i]) * xs;
        double hi = (i == n_nu - 1) ? INFINITY : 0.5 * (nu[i] + nu[i + 1]) * xs;
        F_out[i] = norm * planck_band(lo, hi);
    }
    return RT_OK;
}

rt_status rt_gray_table(const rt_opacity *op, const double *F_nu, double *kappa_gray, double *F_total,
                        double *nu_gray)
{
    if (!op || !op->T || !op->nu || !op->kappa || !F_nu || !kappa_gray || !F_total)
        return fail(nullptr, RT_EINVAL, "rt_gray_table: NULL argument");
    if (op->n_T < 2 || op->n_T > kMaxT || op->n_nu < 1 || op->n_nu > kMaxNu)
        return fail(nullptr, RT_EINVAL, "rt_gray_table: need 2 <= n_T <= 128 and 1 <= n_nu <= 64");
    double Fs = 0.0, nuF = 0.0;
    for (int b = 0; b < op->n_nu; b++) {
        if (!(F_nu[b] >= 0.0) || !isfin(F_nu[b])) return fail(nullptr, RT_EINVAL, "rt_gray_table: bad bin flux");
        Fs += F_nu[b];
        nuF += op->nu[b] * F_nu[b];
    }
    if (!(Fs > 0.0) || !isfin(Fs)) return fail(nullptr, RT_EINVAL, "rt_gray_table: total flux must be positive");
    for (int k = 0; k < op->n_T; k++) {
        double t = 0.0;
        for (int b = 0; b < op->n_nu; b++) t += op->kappa[(long)k * op->n_nu + b] * F_nu[b];
        kappa_gray[k] = t / Fs;
    }
    *F_total = Fs;
    if (nu_gray) *nu_gray = nuF / Fs;
    return RT_OK;
}

rt_status rt_create(rt_ctx **out, const rt_grid *g, int n_nu, void *stream)
{
    if (!out) return fail(nullptr, RT_EINVAL, "rt_create: out is NULL");
    *out = nullptr;
    if (!g || !g->r_face || !g->th_face || !g->ph_face) return fail(nullptr, RT_EINVAL, "rt_create: grid arrays missing");
    if (g->nr < 2 || g->nt < 1 || g->np < 1) return fail(nullptr, RT_EINVAL, "rt_create: need nr >= 2, nt >= 1, np >= 1");
    if (n_nu < 1 || n_nu > kMaxNu) return fail(nullptr, RT_EINVAL, "rt_create: n_nu must be in [1, 64]");
    long n = (long)g->nr * g->nt * g->np;
    if (n > (1L << 40)) return fail(nullptr, RT_EINVAL, "rt_create: grid too large");
    // the ray trace keeps the opacity table in LDS (160 KB per compute unit) and, for the
    // face flux, one radial factor per cell of a column
    if (raytrace_lds_bytes(kMaxT, g->nr, true) > 160 * 1024 || raytrace_lds_bytes(kMaxT, g->nr, false) > 160 * 1024)
        return fail(nullptr, RT_EINVAL, "rt_create: N_r too large for the ray trace (at most 2944 radial cells)");
    for (int i = 0; i < g->nr; i++)
        if (!(g->r_face[i + 1] > g->r_face[i]) || !(g->r_face[i] > 0.0))
            return fail(nullptr, RT_EINVAL, "rt_create: r_face must be positive and increasing");
    for (int j = 0; j < g->nt; j++)
        if (!(g->th_face[j + 1] > g->th_face[j]) || g->th_face[j] < 0.0 || g->th_face[j + 1] > M_PI + 1e-12)
            return fail(nullptr, RT_EINVAL, "rt_create: th_face must increase within [0, pi]");
    for (int k = 0; k < g->np; k++)
        if (!(g->ph_face[k + 1] > g->ph_face[k]))
            return fail(nullptr, RT_EINVAL, "rt_create: ph_face must increase");

    rt_ctx *ctx = new (std::nothrow) rt_ctx();
    if (!ctx) return fail(nullptr, RT_ENOMEM, "rt_create: out of host memory");
    auto bail = [&](rt_status s, const std::string &m) {
        g_err = m;
        rt_destroy(ctx);
        return s;
    };
    if (hipGetDevice(&ctx->device) != hipSuccess) return bail(RT_EDEVICE, "rt_create: no HIP device");
    ctx->stream = (hipStream_t)stream;
    ctx->d = Dims{g->nr, g->nt, g->np, n, (long)g->nr * g->nt};
    ctx->n_nu = n_nu;
    const int nr = g->nr, nt = g->nt, np = g->np;
    ctx->h_rf.assign(g->r_face, g->r_face + nr + 1);
    ctx->h_tf.assign(g->th_face, g->th_face + nt + 1);
    ctx->h_pf.assign(g->ph_face, g->ph_face + np + 1);

    // 1-D geometry factors
    std::vector<double> rf2(nr + 1), rc(nr), dr(nr), shell(nr), volr(nr), hr2(nr), dsr(nr);
    std::vector<double> dcos(nt), sinf(nt + 1), dth(nt), dtc(nt), sinc(nt), tc(nt), dph(np), dpc(np), pc(np);
    const double *rf = g->r_face, *tf = g->th_face, *pf = g->ph_face;
    for (int i = 0; i <= nr; i++) rf2[i] = rf[i] * rf[i];
    for (int i = 0; i < nr; i++) {
        double r0 = rf[i], r1 = rf[i + 1];
        rc[i] = 0.5 * (r0 + r1);
        dr[i] = r1 - r0;
        shell[i] = r1 * r1 * r1 - r0 * r0 * r0;
        volr[i] = shell[i] / 3.0;
        hr2[i] = 0.5 * (r1 * r1 - r0 * r0);
    }
    for (int i = 0; i + 1 < nr; i++) dsr[i] = rc[i + 1] - rc[i];
    {
        double rl = rf[nr], rp = rf[nr - 1];
        double rg = rl * (rl / rp);
        dsr[nr - 1] = 0.5 * (rl + rg) - rc[nr - 1];
    }
    for (int j = 0; j < nt; j++) {
        dcos[j] = std::cos(tf[j]) - std::cos(tf[j + 1]);
        dth[j] = tf[j + 1] - tf[j];
        tc[j] = 0.5 * (tf[j] + tf[j + 1]);
        sinc[j] = std::sin(tc[j]);
    }
    for (int j = 0; j <= nt; j++) sinf[j] = std::sin(tf[j]);
    for (int j = 0; j < nt; j++) dtc[j] = (j + 1 < nt) ? tc[j + 1] - tc[j] : 0.0;
    for (int k = 0; k < np; k++) {
        dph[k] = pf[k + 1] - pf[k];
        pc[k] = 0.5 * (pf[k] + pf[k + 1]);
    }
    for (int k = 0; k < np; k++)
        dpc[k] = (k + 1 < np) ? pc[k + 1] - pc[k] : (pf[np] - pc[np - 1]) + (pc[0] - pf[0]);

    auto up = [&](const std::vector<double> &h) -> const double * {
        double *p = dalloc<double>(ctx, h.size());
        if (!p || hipMemcpy(p, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
            return nullptr;
        return p;
    };
    std::vector<double> rfv(rf, rf + nr + 1);
    Geo &G = ctx->geo;
    if (!(G.rf = up(rfv)) || !(G.rf2 = up(rf2)) || !(G.rc = up(rc)) || !(G.dr = up(dr)) ||
        !(G.shell = up(shell)) || !(G.vol_r = up(volr)) || !(G.hr2 = up(hr2)) || !(G.dsr = up(dsr)) ||
        !(G.dcos = up(dcos)) || !(G.sinf = up(sinf)) || !(G.dth = up(dth)) || !(G.dtc = up(dtc)) ||
        !(G.sinc = up(sinc)) || !(G.dph = up(dph)) || !(G.dpc = up(dpc)))
        return bail(RT_ENOMEM, "rt_create: geometry upload failed");

    // opacity table (max size) and star
    Opac &O = ctx->op;
    double *ot = dalloc<double>(ctx, (size_t)kMaxT * (kMaxNu + 6));
    ctx->F0 = dalloc<double>(ctx, kMaxNu);
    if (!ot || !ctx->F0) return bail(RT_ENOMEM, "rt_create: table allocation failed");
    O.T = ot;
    O.kap = ot + kMaxT;
    O.kP = O.kap + (size_t)kMaxT * kMaxNu;
    O.kR = O.kP + kMaxT;
    O.lnT = O.kR + kMaxT;
    O.lnP = O.lnT + kMaxT;
    O.lnR = O.lnP + kMaxT;
    O.nnu = n_nu;
    O.kconst = 1;

    // fields, system, Krylov vectors
    size_t N = (size_t)n;
    ctx->q = dalloc<double>(ctx, N);
    ctx->S = dalloc<double>(ctx, N);
    ctx->En = dalloc<double>(ctx, N);
    ctx->w = dalloc<double>(ctx, 3 * N);
    ctx->ahat = dalloc<double>(ctx, 3 * N);
    ctx->ahat32 = dalloc<float>(ctx, 3 * N);
    ctx->s = dalloc<double>(ctx, N);
    ctx->b = dalloc<double>(ctx, N);
    ctx->bhat = dalloc<double>(ctx, N);
    ctx->chi = dalloc<double>(ctx, N);
    ctx->y = dalloc<double>(ctx, N);
    ctx->r = dalloc<double>(ctx, N);
    ctx->p0 = dalloc<double>(ctx, N);
    ctx->p1 = dalloc<double>(ctx, N);
    ctx->qv = dalloc<double>(ctx, N);
    ctx->r32 = dalloc<float>(ctx, N);
    ctx->p32a = dalloc<float>(ctx, N);
    ctx->p32b = dalloc<float>(ctx, N);
    ctx->q32 = dalloc<float>(ctx, N);
    ctx->x32 = dalloc<float>(ctx, N);
    ctx->z32 = dalloc<float>(ctx, N);
    ctx->nscale = dalloc<double>(ctx, 2);
    if (!ctx->q || !ctx->S || !ctx->En || !ctx->w || !ctx->ahat || !ctx->ahat32 || !ctx->s || !ctx->b ||
        !ctx->bhat || !ctx->chi || !ctx->y || !ctx->r || !ctx->p0 || !ctx->p1 || !ctx->qv || !ctx->r32 ||
        !ctx->p32a || !ctx->p32b || !ctx->q32 || !ctx->x32 || !ctx->z32 || !ctx->nscale)
        return bail(RT_ENOMEM, "rt_create: out of device memory");

    // block counts (multiples of 8, one share per XCD).  Measured on MI355X at
    // 512x256x512: one block of 256 threads per CU is fastest for both the stencil
    // kernels (each thread keeps all ~20 loads of a segment in flight) and the pure
    // streaming update kernel (fewer, longer streams).
    auto blocks = [&](const char *var, long dflt) {
        const char *e = std::getenv(var);
        long v = e ? std::max(8L, std::atol(e)) : dflt;
        long want = (n + 255) / 256;  // never more blocks than 256-cell portions
        v = std::min(std::max(std::min(v, want), 8L), 65536L);
        return (v + 7) / 8 * 8;
    };
    long nb = blocks("RTMI_BLOCKS", 256);
    ctx->nblk = (int)nb;
    ctx->nblk_upd = (int)blocks("RTMI_BLOCKS_UPD", 256);
    ctx->partials = dalloc<double>(ctx, std::max<long>(nb, ctx->nblk_upd));
    ctx->counter = dalloc<unsigned>(ctx, 4);
    ctx->sc = dalloc<DevScalars>(ctx, 1);
    if (!ctx->partials || !ctx->counter || !ctx->sc) return bail(RT_ENOMEM, "rt_create: out of device memory");
    // direction buffers start at zero: the first CG direction is r + 0 * p_old
    for (void *pz : {(void *)ctx->p0, (void *)ctx->p1})
        if (hipMemset(pz, 0, N * sizeof(double)) != hipSuccess) return bail(RT_EDEVICE, "rt_create: memset failed");
    for (void *pz : {(void *)ctx->p32a, (void *)ctx->p32b})
        if (hipMemset(pz, 0, N * sizeof(float)) != hipSuccess) return bail(RT_EDEVICE, "rt_create: memset failed");
    if (hipMemset(ctx->counter, 0, 4 * sizeof(unsigned)) != hipSuccess ||
        hipMemset(ctx->sc, 0, sizeof(DevScalars)) != hipSuccess)
        return bail(RT_EDEVICE, "rt_create: memset failed");
    if (hipHostMalloc((void **)&ctx->h_sc, sizeof(DevScalars), hipHostMallocDefault) != hipSuccess)
        return bail(RT_ENOMEM, "rt_create: pinned allocation failed");
    std::memset(ctx->h_sc, 0, sizeof(DevScalars));
    for (auto &e : ctx->ev)
        if (hipEventCreate(&e) != hipSuccess) return bail(RT_EDEVICE, "rt_create: event creation failed");
    raytrace_prepare();
    *out = ctx;
    return RT_OK;
}

void rt_destroy(rt_ctx *ctx)
{
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    for (auto &g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    for (void *p : ctx->allocs) (void)hipFree(p);
    delete ctx->mg;
    if (ctx->h_sc) (void)hipHostFree(ctx->h_sc);
    for (auto &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    delete ctx;
}

rt_status rt_set_opacity(rt_ctx *ctx, const rt_opacity *op)
{
    if (!ctx) return fail(nullptr, RT_EINVAL, "context is NULL");
    RT_CHECK(ctx, op && op->T && op->kappa && op->kappa_P && op->kappa_R, "opacity arrays missing");
    RT_CHECK(ctx, op->n_T >= 2 && op->n_T <= kMaxT, "n_T must be in [2, 128]");
    RT_CHECK(ctx, op->n_nu == ctx->n_nu, "opacity n_nu differs from the context's");
    const int nT = op->n_T, nnu = op->n_nu;
    for (int k = 0; k < nT; k++) {
        RT_CHECK(ctx, op->T[k] > 0.0 && (k == 0 || op->T[k] > op->T[k - 1]), "table T must be positive and increasing");
        RT_CHECK(ctx, op->kappa_P[k] > 0.0 && op->kappa_R[k] > 0.0 && isfin(op->kappa_P[k]) && isfin(op->kappa_R[k]),
                 "mean opacities must be positive");
        for (int b = 0; b < nnu; b++)
            RT_CHECK(ctx, op->kappa[(size_t)k * nnu + b] >= 0.0 && isfin(op->kappa[(size_t)k * nnu + b]),
                     "kappa_nu must be finite and >= 0");
    }
    std::vector<double> pack;
    pack.reserve((size_t)nT * (nnu + 3) + 1);
    pack.push_back(nT);
    pack.insert(pack.end(), op->T, op->T + nT);
    pack.insert(pack.end(), op->kappa, op->kappa + (size_t)nT * nnu);
    pack.insert(pack.end(), op->kappa_P, op->kappa_P + nT);
    pack.insert(pack.end(), op->kappa_R, op->kappa_R + nT);
    if (ctx->have_opac && pack == ctx->h_opac) return RT_OK;
    std::vector<double> lnT(nT), lnP(nT), lnR(nT);
    for (int k = 0; k < nT; k++) {
        lnT[k] = std::log(op->T[k]);
        lnP[k] = std::log(op->kappa_P[k]);
        lnR[k] = std::log(op->kappa_R[k]);
    }
    RT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    Opac &O = ctx->op;
    RT_HIP(ctx, hipMemcpy((void *)O.T, op->T, nT * sizeof(double), hipMemcpyHostToDevice));
    RT_HIP(ctx, hipMemcpy((void *)O.kap, op->kappa, (size_t)nT * nnu * sizeof(double), hipMemcpyHostToDevice));
    RT_HIP(ctx, hipMemcpy((void *)O.kP, op->kappa_P, nT * sizeof(double), hipMemcpyHostToDevice));
    RT_HIP(ctx, hipMemcpy((void *)O.kR, op->kappa_R, nT * sizeof(double), hipMemcpyHostToDevice));
    RT_HIP(ctx, hipMemcpy((void *)O.lnT, lnT.data(), nT * sizeof(double), hipMemcpyHostToDevice));
    RT_HIP(ctx, hipMemcpy((void *)O.lnP, lnP.data(), nT * sizeof(double), hipMemcpyHostToDevice));
    RT_HIP(ctx, hipMemcpy((void *)O.lnR, lnR.data(), nT * sizeof(double), hipMemcpyHostToDevice));
    O.nT = nT;
    // the leading temperature rows whose kappa_nu equal row 0's bit for bit (below dust
    // sublimation kappa_nu does not depend on T): where every node a column's cells use
    // lies in them, the ray trace takes kappa_nu from row 0
    int kc = 1;
    while (kc < nT && std::equal(op->kappa + (size_t)kc * nnu, op->kappa + (size_t)(kc + 1) * nnu, op->kappa)) kc++;
    O.kconst = kc;
    ctx->nT = nT;
    ctx->h_opac.swap(pack);
    ctx->have_opac = true;
    return RT_OK;
}

rt_status rt_set_star(rt_ctx *ctx, const rt_star *st)
{
    if (!ctx) return fail(nullptr, RT_EINVAL, "context is NULL");
    RT_CHECK(ctx, st && st->F_nu, "star flux array missing");
    RT_CHECK(ctx, st->R_star > 0.0 && isfin(st->R_star), "R_star must be positive");
    RT_CHECK(ctx, st->R_star <= ctx->h_rf[0], "R_star must not exceed the inner radial face");
    for (int b = 0; b < ctx->n_nu; b++)
        RT_CHECK(ctx, st->F_nu[b] >= 0.0 && isfin(st->F_nu[b]), "F_nu must be finite and >= 0");
    std::vector<double> pack(st->F_nu, st->F_nu + ctx->n_nu);
    pack.push_back(st->R_star);
    pack.push_back(st->T_star);
    if (ctx->have_star && pack == ctx->h_star) return RT_OK;
    RT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    RT_HIP(ctx, hipMemcpy(ctx->F0, st->F_nu, ctx->n_nu * sizeof(double), hipMemcpyHostToDevice));
    ctx->R_star = st->R_star;
    ctx->T_star = st->T_star;
    ctx->h_star.swap(pack);
    ctx->have_star = true;
    return RT_OK;
}

rt_status rt_raytrace(rt_ctx *ctx, const rt_opacity *op, const rt_star *st, const double *rho, const double *T,
                      double *q_star, double *S_abs, double *F_face, double *F_face_nu)
{
    if (!ctx) return fail(nullptr, RT_EINVAL, "context is NULL");
    if (op) { rt_status s = rt_set_opacity(ctx, op); if (s) return s; }
    if (st) { rt_status s = rt_set_star(ctx, st); if (s) return s; }
    RT_CHECK(ctx, ctx->have_opac, "no opacity table on the context");
    RT_CHECK(ctx, ctx->have_star, "no star on the context");
    RT_CHECK(ctx, rho && T && q_star && S_abs, "rt_raytrace: NULL field pointer");
    launch_raytrace(ctx->d, ctx->op, ctx->geo, ctx->F0, ctx->R_star * ctx->R_star, rho, T, q_star, S_abs, F_face,
                    F_face_nu, ctx->stream);
    RT_HIP(ctx, hipGetLastError());
    return RT_OK;
}

rt_status rt_raytrace_mapped(rt_ctx *ctx, int mapping, const double *rho, const double *T, double *q_star,
                             double *S_abs)
{
    if (!ctx) return fail(nullptr, RT_EINVAL, "context is NULL");
    RT_CHECK(ctx, ctx->have_opac, "no opacity table on the context");
    RT_CHECK(ctx, ctx->have_star, "no star on the context");
    RT_CHECK(ctx, rho && T && q_star && S_abs, "rt_raytrace_mapped: NULL field pointer");
    RT_CHECK(ctx, mapping == RT_LANES_BINS || mapping == RT_LANES_CELLS, "mapping must be an rt_raytrace_mapping");
    if (mapping == RT_LANES_CELLS)
        launch_raytrace_r(ctx->d, ctx->op, ctx->geo, ctx->F0, ctx->R_star * ctx->R_star, rho, T, q_star, S_abs,
                          ctx->stream);
    else
        launch_raytrace_bins(ctx->d, ctx->op, ctx->geo, ctx->F0, ctx->R_star * ctx->R_star, rho, T, q_star, S_abs,
                             nullptr, nullptr, ctx->stream);
    RT_HIP(ctx, hipGetLastError());
    return RT_OK;
}

rt_status rt_energy(rt_ctx *ctx, const rt_opacity *op, const rt_fld_params *p, const double *T, const double *S_abs,
                    double *E)
{
    if (!ctx) return fail(nullptr, RT_EINVAL, "context is NULL");
    if (op) { rt_status s = rt_set_opacity(ctx, op); if (s) return s; }
    RT_CHECK(ctx, ctx->have_opac, "no opacity table on the context");
    if (rt_status s = check_fld(ctx, p)) return s;
    RT_CHECK(ctx, T && S_abs && E, "rt_energy: NULL field pointer");
    launch_energy(ctx->d, ctx->op, T, S_abs, p->E_floor, E, ctx->stream);
    RT_HIP(ctx, hipGetLastError());
    return RT_OK;
}

rt_status rt_fld_assemble(rt_ctx *ctx, const rt_opacity *op, const rt_fld_params *p, const double *rho,
                          const double *T, const double *E_n, const double *q_star, const double *Q_plus,
                          rt_system *sys)
{
    if (!ctx) return fail(nullptr, RT_EINVAL, "context is NULL");
    if (op) { rt_status s = rt_set_opacity(ctx, op); if (s) return s; }
    RT_CHECK(ctx, ctx->have_opac, "no opacity table on the context");
    if (rt_status s = check_fld(ctx, p)) return s;
    RT_CHECK(ctx, rho && T && E_n && q_star, "rt_fld_assemble: NULL field pointer");
    std::vector<double> Tt(ctx->h_opac.begin() + 1, ctx->h_opac.begin() + 1 + ctx->nT);
    std::vector<double> kR(ctx->h_opac.end() - ctx->nT, ctx->h_opac.end());
    double kR_bc = host_mean(Tt, kR, p->T_bc);
    double Eb = kA * std::pow(p->T_bc, 4);
    ctx->Eb = Eb;
    launch_assemble(ctx->d, ctx->geo, ctx->op, rho, T, E_n, q_star, Q_plus, p->c_V, p->dt, Eb, kR_bc, ctx->chi,
                    ctx->w, ctx->s, ctx->b, ctx->bhat, ctx->ahat, ctx->ahat32, ctx->stream);
    RT_HIP(ctx, hipGetLastError());
    ctx->have_system = true;
    ctx->rb_ready = false;
    ctx->ln_ready = false;
    if (ctx->mg) ctx->mg->ready = false;
    if (sys) {
        sys->n = ctx->d.n;
        sys->ahat = ctx->ahat;
        sys->ahat32 = ctx->ahat32;
        sys->s = ctx->s;
        sys->bhat = ctx->bhat;
        sys->w = ctx->w;
        sys->chi = ctx->chi;
    }
    return RT_OK;
}

rt_status rt_spmv(rt_ctx *ctx, const double *x, double *y)
{
    if (!ctx) return fail(nullptr, RT_EINVAL, "context is NULL");
    RT_CHECK(ctx, ctx->have_system, "no assembled system");
    RT_CHECK(ctx, x && y && x != y, "rt_spmv: bad vectors");
    launch_spmv(ctx->d, ctx->nblk, ctx->ahat, x, y, ctx->stream);
    RT_HIP(ctx, hipGetLastError());
    return RT_OK;
}

}  // extern "C"

namespace {

struct Clock {
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double ms() const
    {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

// Adds the device times of the sampled iteration (events 8, 9, 10; 11 between the red
// and black passes of a reduced solve) to the stats.
void add_kernel_sample(rt_ctx *ctx, rt_solve_stats *st, bool rb = false)
{
    float a = 0.f, b = 0.f, c = 0.f;
    if (hipEventElapsedTime(&a, ctx->ev[8], ctx->ev[9]) != hipSuccess) return;
    if (hipEventElapsedTime(&b, ctx->ev[9], ctx->ev[10]) != hipSuccess) return;
    if (rb && hipEventElapsedTime(&c, ctx->ev[11], ctx->ev[9]) != hipSuccess) return;
    int n = st->kernel_samples;
    st->ms_dir = (st->ms_dir * n + a) / (n + 1);
    st->ms_upd = (st->ms_upd * n + b) / (n + 1);
    st->ms_black = (st->ms_black * n + c) / (n + 1);
    st->kernel_samples = n + 1;
}

// Grids up to this many cells run their Krylov iterations from HIP graphs by default:
// their kernels take a few microseconds, so launches dominate.
constexpr long kGraphCells = 1L << 22;
constexpr size_t kMaxGraphs = 16;

bool use_graphs(const rt_ctx *ctx, const rt_solve_opts *o)
{
    return o->launch == RT_LAUNCH_GRAPH ||
           ((o->launch == RT_LAUNCH_AUTO || o->launch == RT_LAUNCH_BLOCK) && ctx->d.n <= kGraphCells);
}

// The reduced float64 solve runs in one workgroup (launches of up to kBlockChunk
// iterations, a few tens of ms each).
constexpr int kBlockChunk = 16384;

bool use_block(const rt_solve_opts *o, const Dims &dh)
{
    return (o->launch == RT_LAUNCH_AUTO || o->launch == RT_LAUNCH_BLOCK) && rb_block_cpt(dh) > 0;
}

// Enqueues m Krylov iterations on ctx->stream, each launched by iter(pold, pnew, stream,
// ev, k) (ev: the events that time the first iteration's kernels, or NULL; k: the
// iteration's index in the chunk), swapping the direction buffers after each.  With
// graphs the m launches are captured once per (kind, pold, m) on a private stream and
// the instantiated graph is replayed (the kernels read every scalar from device memory,
// so a replay is the same work as the launches); *sampled tells whether the events were
// recorded.
template <typename T, typename F>
rt_status run_iters(rt_ctx *ctx, const rt_solve_opts *o, int kind, int m, T *&pold, T *&pnew, F &&iter,
                    bool *sampled)
{
    hipGraphExec_t ex = nullptr;
    if (use_graphs(ctx, o))
        for (const auto &g : ctx->graphs)
            if (g.kind == kind && g.pold == (const void *)pold && g.m == m) ex = g.exec;
    // chunk lengths other than the polling interval (the last chunk before max_iter) are
    // rare: at most kMaxGraphs graphs are kept, later new shapes launch directly
    if (!ex && (!use_graphs(ctx, o) || ctx->graphs.size() >= kMaxGraphs)) {
        for (int k = 0; k < m; k++) {
            iter(pold, pnew, ctx->stream, k == 0 ? &ctx->ev[8] : nullptr, k);
            std::swap(pold, pnew);
        }
        *sampled = true;
        return RT_OK;
    }
    *sampled = false;
    if (!ex) {
        if (!ctx->cap_stream) RT_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        RT_HIP(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
        T *a = pold, *b = pnew;
        for (int k = 0; k < m; k++) {
            iter(a, b, ctx->cap_stream, nullptr, k);
            std::swap(a, b);
        }
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &g);
        if (ec != hipSuccess || !g) return fail(ctx, RT_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
        const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) return fail(ctx, RT_EDEVICE, std::string("graph instantiation: ") + hipGetErrorString(ei));
        ctx->graphs.push_back({kind, (const void *)pold, m, ex});
    }
    RT_HIP(ctx, hipGraphLaunch(ex, ctx->stream));
    if (m % 2) std::swap(pold, pnew);
    return RT_OK;
}

// ||bhat||^2 on the device, read back.
rt_status norm_b(rt_ctx *ctx, double &bb)
{
    launch_norm2(ctx->d, ctx->nblk, ctx->bhat, ctx->partials, ctx->counter, ctx->sc, ctx->stream);
    RT_HIP(ctx, hipGetLastError());
    if (rt_status s = read_scalars(ctx)) return s;
    bb = ctx->h_sc->res2;
    return RT_OK;
}

// Zeroes the float64 and float32 direction buffers.  Every CG restart forms p = r +
// 0 * p_old, which a non-finite p_old would poison, so a solve that continues after a
// non-finite exit (the learned solve's fallback) or the next call after a failed one
// starts from zero directions again, as at creation.
rt_status reset_directions(rt_ctx *ctx)
{
    const size_t N = (size_t)ctx->d.n;
    for (void *pz : {(void *)ctx->p0, (void *)ctx->p1})
        RT_HIP(ctx, hipMemsetAsync(pz, 0, N * sizeof(double), ctx->stream));
    for (void *pz : {(void *)ctx->p32a, (void *)ctx->p32b})
        RT_HIP(ctx, hipMemsetAsync(pz, 0, N * sizeof(float), ctx->stream));
    return RT_OK;
}

// Plain float64 CG on A^ (the method; also the fallback of the other modes and the
// reference they are checked against).
rt_status solve_fp64(rt_ctx *ctx, const rt_solve_opts *o, rt_solve_stats *st, double bb)
{
    const Dims &d = ctx->d;
    hipStream_t s = ctx->stream;
    DevScalars *h = ctx->h_sc;
    h->thresh2 = o->tol * o->tol * bb;
    h->done = 0;
    h->iters = 0;
    h->beta = 0.0;
    if (rt_status e = write_scalars(ctx)) return e;
    launch_resid(d, ctx->nblk, ctx->ahat, ctx->bhat, ctx->y, ctx->r, ctx->partials, ctx->counter,
                 ctx->sc, 1, s);
    if (rt_status e = read_scalars(ctx)) return e;
    double *pold = ctx->p0, *pnew = ctx->p1;
    const int every = o->check_every > 0 ? o->check_every : 32;
    rt_status status = RT_OK;
    double res = std::sqrt(h->res2 / bb);  // true residual of the start guess
    for (;;) {
        st->relres = res;
        if (!isfin(res)) { status = RT_ENONFINITE; break; }
        if (res <= o->tol) break;
        if (h->iters >= o->max_iter) { status = RT_ENOCONV; break; }
        int m = std::min(every, o->max_iter - h->iters);
        int it_before = h->iters;
        bool sampled = false;
        if (rt_status e = run_iters(ctx, o, 0, m, pold, pnew, [&](double *a, double *b, hipStream_t ss, const hipEvent_t *ev, int k) {
                launch_cg_iter64(d, ctx->nblk, ctx->nblk_upd, ctx->ahat, ctx->y, ctx->r, a, b, ctx->qv, ctx->partials,
                                 ctx->counter, ctx->sc, ss, ev, k & 1);
            }, &sampled))
            return e;
        RT_HIP(ctx, hipGetLastError());
        if (rt_status e = read_scalars(ctx)) return e;
        if (sampled) add_kernel_sample(ctx, st);
        if ((h->iters - it_before) % 2 != m % 2) std::swap(pold, pnew);  // kernels that exited early
        if (!isfin(h->rr)) { status = RT_ENONFINITE; st->relres = NAN; break; }
        if (h->done || h->iters >= o->max_iter) {
            // the recurrence met the tolerance (or the budget ran out): judge by the true
            // residual, and restart CG from it if it is still above the tolerance
            launch_resid(d, ctx->nblk, ctx->ahat, ctx->bhat, ctx->y, ctx->r, ctx->partials,
                         ctx->counter, ctx->sc, 1, s);
            if (rt_status e = read_scalars(ctx)) return e;
            res = std::sqrt(h->res2 / bb);
        }
    }
    st->iters = h->iters;
    return status;
}

// Mixed precision: CG iterations in float32 (operator, vectors and recurrences) with
// float64 dot products, and "reliable updates" in float64: whenever the float32
// recurrence residual has fallen by a factor 10 since the last update (or claims
// convergence), the float32 partial solution is folded into the float64 solution y,
// the true residual b - A y is recomputed in float64 and replaces the float32 one,
// and CG continues along its current direction.  Convergence is judged only on the
// float64 residual.
rt_status solve_mixed(rt_ctx *ctx, const rt_solve_opts *o, rt_solve_stats *st, double bb)
{
    const Dims &d = ctx->d;
    hipStream_t s = ctx->stream;
    DevScalars *h = ctx->h_sc;
    const double delta2 = 0.01;
    // Precision guard.  CG needs about 1.15 sqrt(cond) iterations per tenfold residual
    // reduction, so a float32 cycle that has not reached its tenfold drop after kCycle
    // iterations means cond(A^) eps32 is no longer small (cond above ~3e6): float32
    // iterations then lose conjugacy and need several times the float64 count.  Such a
    // cycle is folded in and float64 CG finishes from that iterate; so does a solve
    // whose cycles twice in a row fail to halve the true residual.
    const int kCycle = 2048;
    h->iters = 0;
    h->done = 0;
    h->beta = 0.0;
    h->thresh2 = o->tol * o->tol * bb;
    if (rt_status e = write_scalars(ctx)) return e;
    const int every = o->check_every > 0 ? o->check_every : 32;
    launch_resid(d, ctx->nblk, ctx->ahat, ctx->bhat, ctx->y, ctx->r, ctx->partials, ctx->counter,
                 ctx->sc, 0, s);
    launch_reliable(d, ctx->nblk, ctx->r, ctx->r32, ctx->x32, ctx->partials, ctx->counter, ctx->sc, 1, s);
    if (rt_status e = read_scalars(ctx)) return e;
    double res = std::sqrt(h->res2 / bb), rr_ref = h->res2;
    float *pold = ctx->p32a, *pnew = ctx->p32b;
    rt_status status = RT_OK;
    int cycle_start = 0, bad = 0;
    bool fallback = false;
    for (;;) {
        st->relres = res;
        if (!isfin(res)) { status = RT_ENONFINITE; break; }
        if (res <= o->tol) break;
        if (h->iters >= o->max_iter) { status = RT_ENOCONV; break; }
        if (bad >= 2) { fallback = true; break; }
        int m = std::min(every, o->max_iter - h->iters);
        int it_before = h->iters;
        bool sampled = false;
        if (rt_status e = run_iters(ctx, o, 1, m, pold, pnew, [&](float *a, float *b, hipStream_t ss, const hipEvent_t *ev, int k) {
                launch_cg_iter32(d, ctx->nblk, ctx->nblk_upd, ctx->ahat32, ctx->x32, ctx->r32, a, b, ctx->q32,
                                 ctx->partials, ctx->counter, ctx->sc, ss, ev, k & 1);
            }, &sampled))
            return e;
        RT_HIP(ctx, hipGetLastError());
        if (rt_status e = read_scalars(ctx)) return e;
        if (sampled) add_kernel_sample(ctx, st);
        if ((h->iters - it_before) % 2 != m % 2) std::swap(pold, pnew);  // kernels that exited early
        if (!isfin(h->rr)) { status = RT_ENONFINITE; st->relres = NAN; break; }
        const bool capped = h->iters - cycle_start >= kCycle;
        if (h->done || h->rr <= delta2 * rr_ref || h->iters >= o->max_iter || capped) {
            launch_fold(d.n, ctx->x32, ctx->y, s);
            launch_resid(d, ctx->nblk, ctx->ahat, ctx->bhat, ctx->y, ctx->r, ctx->partials,
                         ctx->counter, ctx->sc, 0, s);
            launch_reliable(d, ctx->nblk, ctx->r, ctx->r32, ctx->x32, ctx->partials, ctx->counter,
                            ctx->sc, 0, s);
            RT_HIP(ctx, hipGetLastError());
            if (rt_status e = read_scalars(ctx)) return e;
            const double res_new = std::sqrt(h->res2 / bb);
            bad = (res_new > 0.5 * res) ? bad + 1 : 0;
            if (capped && res_new > o->tol) bad = 2;
            res = res_new;
            rr_ref = h->res2;
            cycle_start = h->iters;
            st->outer_iters++;
        }
    }
    st->iters = h->iters;
    if (fallback) {
        st->fallback = 1;
        rt_solve_stats s64{};
        rt_solve_opts o64 = *o;
        o64.mode = RT_SOLVE_FP64;
        o64.max_iter = std::max(1, o->max_iter - st->iters);
        status = solve_fp64(ctx, &o64, &s64, bb);
        st->iters += s64.iters;
        st->relres = s64.relres;
    }
    return status;
}

// The red-black reduced system (k_krylov.hip): CG on S = I - B^T B over the black
// cells, then y_r = b_r - B y_b.  Needs N_r even (compact colour halves per radial
// row) and N_phi even or 1 (the periodic seam joins opposite colours).
bool rb_possible(const rt_ctx *ctx)
{
    return ctx->d.nr % 2 == 0 && (ctx->d.np == 1 || ctx->d.np % 2 == 0) && ctx->d.nr >= 2;
}

// Colour split of the current operator (once per assembled system), the reduced
// right-hand side bb = b_b - B^T b_r and b_r in `rhs` ([bb | b_r], n/2 each), and y_b
// gathered from the natural start vector ctx->y.  `tmp` (n/2) holds b_b on the way.
rt_status rb_prepare(rt_ctx *ctx, double *rhs, double *yb, double *tmp)
{
    const Dims &d = ctx->d;
    const long n = d.n, nh = n / 2;
    if (!ctx->rb_a) {
        ctx->rb_a = dalloc<double>(ctx, 3 * n);
        ctx->rb_a32 = dalloc<float>(ctx, 3 * n);
        if (!ctx->rb_a || !ctx->rb_a32) return fail(ctx, RT_ENOMEM, "red-black split: out of device memory");
    }
    hipStream_t s = ctx->stream;
    if (!ctx->rb_ready) {
        launch_rb_split(d, ctx->ahat, ctx->rb_a, ctx->rb_a32, s);
        ctx->rb_ready = true;
    }
    const Dims dh = rb_half(d);
    launch_rb_gather(d, ctx->bhat, tmp, rhs + nh, s);
    launch_rb_black_apply(dh, ctx->nblk, ctx->rb_a, rhs + nh, tmp, nullptr, -1.0, rhs, ctx->partials, ctx->counter,
                          ctx->sc, 0, s);
    launch_rb_gather(d, ctx->y, yb, nullptr, s);
    RT_HIP(ctx, hipGetLastError());
    return RT_OK;
}

// r_b = bb - S y_b in float64 (t_r receives B y_b); restart as in k_resid.
void rb_resid(rt_ctx *ctx, const double *rhs, const double *yb, double *rb, double *tr, int restart)
{
    const Dims dh = rb_half(ctx->d);
    launch_rb_red_apply(dh, ctx->nblk, ctx->rb_a, yb, nullptr, 1.0, tr, ctx->stream);
    launch_rb_black_apply(dh, ctx->nblk, ctx->rb_a, tr, rhs, yb, 1.0, rb, ctx->partials, ctx->counter, ctx->sc,
                          restart, ctx->stream);
}

// y_r = b_r - B y_b, and the natural solution ctx->y from both halves.
rt_status rb_finish(rt_ctx *ctx, const double *rhs, const double *yb, double *yr)
{
    const Dims dh = rb_half(ctx->d);
    const long nh = ctx->d.n / 2;
    launch_rb_red_apply(dh, ctx->nblk, ctx->rb_a, yb, rhs + nh, -1.0, yr, ctx->stream);
    launch_rb_scatter(ctx->d, yb, yr, ctx->y, ctx->stream);
    RT_HIP(ctx, hipGetLastError());
    return RT_OK;
}

// Float64 CG on the reduced system (the same stopping test as solve_fp64: the true
// residual of S is the residual of A^ after the back substitution).  Workspace: the
// halves of the full-system Krylov vectors.
rt_status solve_fp64_rb(rt_ctx *ctx, const rt_solve_opts *o, rt_solve_stats *st, double bb)
{
    const Dims dh = rb_half(ctx->d);
    const long nh = dh.n;
    DevScalars *h = ctx->h_sc;
    double *rb = ctx->r, *tr = ctx->r + nh, *pold = ctx->p0, *pnew = ctx->p0 + nh;
    double *qb = ctx->qv, *yb = ctx->qv + nh, *rhs = ctx->p1;
    if (rt_status e = rb_prepare(ctx, rhs, yb, rb)) return e;
    h->thresh2 = o->tol * o->tol * bb;
    h->done = 0;
    h->iters = 0;
    h->beta = 0.0;
    if (rt_status e = write_scalars(ctx)) return e;
    rb_resid(ctx, rhs, yb, rb, tr, 1);
    if (rt_status e = read_scalars(ctx)) return e;
    const int every = o->check_every > 0 ? o->check_every : 32;
    const bool block = use_block(o, dh);
    rt_status status = RT_OK;
    double res = std::sqrt(h->res2 / bb);
    for (;;) {
        st->relres = res;
        if (!isfin(res)) { status = RT_ENONFINITE; break; }
        if (res <= o->tol) break;
        if (h->iters >= o->max_iter) { status = RT_ENOCONV; break; }
        if (block) {  // one direction buffer: the kernel updates p in place
            const int m = std::min(kBlockChunk, o->max_iter - h->iters);
            if (!launch_rb_cg_block(dh, ctx->rb_a, yb, rb, pold, m, ctx->sc, ctx->stream))
                return fail(ctx, RT_EDEVICE, "one-workgroup CG: grid too large");
            RT_HIP(ctx, hipGetLastError());
            if (rt_status e = read_scalars(ctx)) return e;
        } else {
            int m = std::min(every, o->max_iter - h->iters);
            int it_before = h->iters;
            bool sampled = false;
            if (rt_status e = run_iters(ctx, o, 2, m, pold, pnew, [&](double *a, double *b, hipStream_t ss, const hipEvent_t *ev, int) {
                    launch_rb_iter64(dh, ctx->nblk, ctx->nblk_upd, ctx->rb_a, yb, rb, a, b, qb, tr, ctx->partials,
                                     ctx->counter, ctx->sc, ss, ev);
                }, &sampled))
                return e;
            RT_HIP(ctx, hipGetLastError());
            if (rt_status e = read_scalars(ctx)) return e;
            if (sampled) add_kernel_sample(ctx, st, true);
            if ((h->iters - it_before) % 2 != m % 2) std::swap(pold, pnew);  // kernels that exited early
        }
        if (!isfin(h->rr)) { status = RT_ENONFINITE; st->relres = NAN; break; }
        if (h->done || h->iters >= o->max_iter) {
            rb_resid(ctx, rhs, yb, rb, tr, 1);
            if (rt_status e = read_scalars(ctx)) return e;
            res = std::sqrt(h->res2 / bb);
        }
    }
    st->iters = h->iters;
    st->reduced = 1;
    if (rt_status e = rb_finish(ctx, rhs, yb, tr)) return e;
    return status;
}

// Mixed precision on the reduced system: float32 CG on S with float64 reliable updates
// (the scheme and guards of solve_mixed, iterations counted on S); a guard that trips
// hands over to float64 CG on S from the current iterate.
rt_status solve_mixed_rb(rt_ctx *ctx, const rt_solve_opts *o, rt_solve_stats *st, double bb)
{
    const Dims dh = rb_half(ctx->d);
    const long nh = dh.n;
    hipStream_t s = ctx->stream;
    DevScalars *h = ctx->h_sc;
    double *rb = ctx->r, *tr = ctx->r + nh, *yb = ctx->qv + nh, *rhs = ctx->p1;
    float *r32 = ctx->r32, *t32 = ctx->r32 + nh, *q32 = ctx->q32, *x32 = ctx->q32 + nh;
    float *pold = ctx->p32a, *pnew = ctx->p32a + nh;
    if (rt_status e = rb_prepare(ctx, rhs, yb, rb)) return e;
    const double delta2 = 0.01;
    const int kCycle = 2048;
    h->iters = 0;
    h->done = 0;
    h->beta = 0.0;
    h->thresh2 = o->tol * o->tol * bb;
    if (rt_status e = write_scalars(ctx)) return e;
    const int every = o->check_every > 0 ? o->check_every : 32;
    rb_resid(ctx, rhs, yb, rb, tr, 0);
    launch_reliable(dh, ctx->nblk, rb, r32, x32, ctx->partials, ctx->counter, ctx->sc, 1, s);
    if (rt_status e = read_scalars(ctx)) return e;
    double res = std::sqrt(h->res2 / bb), rr_ref = h->res2;
    rt_status status = RT_OK;
    int cycle_start = 0, bad = 0;
    bool fallback = false;
    for (;;) {
        st->relres = res;
        if (!isfin(res)) { status = RT_ENONFINITE; break; }
        if (res <= o->tol) break;
        if (h->iters >= o->max_iter) { status = RT_ENOCONV; break; }
        if (bad >= 2) { fallback = true; break; }
        int m = std::min(every, o->max_iter - h->iters);
        int it_before = h->iters;
        bool sampled = false;
        if (rt_status e = run_iters(ctx, o, 3, m, pold, pnew, [&](float *a, float *b, hipStream_t ss, const hipEvent_t *ev, int) {
                launch_rb_iter32(dh, ctx->nblk, ctx->nblk_upd, ctx->rb_a32, x32, r32, a, b, q32, t32, ctx->partials,
                                 ctx->counter, ctx->sc, ss, ev);
            }, &sampled))
            return e;
        RT_HIP(ctx, hipGetLastError());
        if (rt_status e = read_scalars(ctx)) return e;
        if (sampled) add_kernel_sample(ctx, st, true);
        if ((h->iters - it_before) % 2 != m % 2) std::swap(pold, pnew);  // kernels that exited early
        if (!isfin(h->rr)) { status = RT_ENONFINITE; st->relres = NAN; break; }
        const bool capped = h->iters - cycle_start >= kCycle;
        if (h->done || h->rr <= delta2 * rr_ref || h->iters >= o->max_iter || capped) {
            launch_fold(nh, x32, yb, s);
            rb_resid(ctx, rhs, yb, rb, tr, 0);
            launch_reliable(dh, ctx->nblk, rb, r32, x32, ctx->partials, ctx->counter, ctx->sc, 0, s);
            RT_HIP(ctx, hipGetLastError());
            if (rt_status e = read_scalars(ctx)) return e;
            const double res_new = std::sqrt(h->res2 / bb);
            bad = (res_new > 0.5 * res) ? bad + 1 : 0;
            if (capped && res_new > o->tol) bad = 2;
            res = res_new;
            rr_ref = h->res2;
            cycle_start = h->iters;
            st->outer_iters++;
        }
    }
    st->iters = h->iters;
    st->reduced = 1;
    if (rt_status e = rb_finish(ctx, rhs, yb, tr)) return e;
    if (fallback) {
        st->fallback = 1;
        rt_solve_stats s64{};
        rt_solve_opts o64 = *o;
        o64.mode = RT_SOLVE_FP64;
        o64.max_iter = std::max(1, o->max_iter - st->iters);
        status = solve_fp64_rb(ctx, &o64, &s64, bb);
        st->iters += s64.iters;
        st->relres = s64.relres;
    }
    return status;
}

// Float64 CG preconditioned by the radial-line block Jacobi (the comparator for the
// paper's block-Jacobi class): the same stopping test on the true residual as solve_fp64.
rt_status solve_fp64_line(rt_ctx *ctx, const rt_solve_opts *o, rt_solve_stats *st, double bb)
{
    const Dims &d = ctx->d;
    const long n = d.n;
    hipStream_t s = ctx->stream;
    DevScalars *h = ctx->h_sc;
    if (!ctx->ln_c) {
        ctx->ln_c = dalloc<double>(ctx, n);
        ctx->ln_im = dalloc<double>(ctx, n);
        ctx->ln_z = dalloc<double>(ctx, n);
        if (!ctx->ln_c || !ctx->ln_im || !ctx->ln_z) return fail(ctx, RT_ENOMEM, "line preconditioner: out of device memory");
    }
    if (!ctx->ln_ready) {
        launch_line_factor(d, ctx->nblk, ctx->ahat, ctx->ln_c, ctx->ln_im, s);
        ctx->ln_ready = true;
    }
    h->thresh2 = o->tol * o->tol * bb;
    h->done = 0;
    h->iters = 0;
    h->beta = 0.0;
    if (rt_status e = write_scalars(ctx)) return e;
    launch_resid(d, ctx->nblk, ctx->ahat, ctx->bhat, ctx->y, ctx->r, ctx->partials, ctx->counter, ctx->sc, 1, s);
    if (rt_status e = read_scalars(ctx)) return e;
    double *pold = ctx->p0, *pnew = ctx->p1;
    const int every = o->check_every > 0 ? o->check_every : 32;
    rt_status status = RT_OK;
    double res = std::sqrt(h->res2 / bb);
    bool restart = true;
    for (;;) {
        st->relres = res;
        if (!isfin(res)) { status = RT_ENONFINITE; break; }
        if (res <= o->tol) break;
        if (h->iters >= o->max_iter) { status = RT_ENOCONV; break; }
        int m = std::min(every, o->max_iter - h->iters);
        int it_before = h->iters;
        for (int k = 0; k < m; k++) {
            launch_pcg_line_iter(d, ctx->nblk, ctx->nblk_upd, ctx->ahat, ctx->ln_c, ctx->ln_im, ctx->y, ctx->r,
                                 ctx->ln_z, pold, pnew, ctx->qv, ctx->partials, ctx->counter, ctx->sc,
                                 restart && k == 0, s, k == 0 ? &ctx->ev[8] : nullptr);
            std::swap(pold, pnew);
        }
        restart = false;
        RT_HIP(ctx, hipGetLastError());
        if (rt_status e = read_scalars(ctx)) return e;
        add_kernel_sample(ctx, st, true);
        if ((h->iters - it_before) % 2 != m % 2) std::swap(pold, pnew);  // kernels that exited early
        if (!isfin(h->res2)) { status = RT_ENONFINITE; st->relres = NAN; break; }
        if (h->done || h->iters >= o->max_iter) {
            launch_resid(d, ctx->nblk, ctx->ahat, ctx->bhat, ctx->y, ctx->r, ctx->partials, ctx->counter,
                         ctx->sc, 1, s);
            if (rt_status e = read_scalars(ctx)) return e;
            res = std::sqrt(h->res2 / bb);
            restart = true;
        }
    }
    st->iters = h->iters;
    return status;
}

// Multigrid hierarchy of the current system: allocated at the first use (levels from
// the grid's theta and phi sizes down to one radial line), set up once per assembled
// system.
constexpr float kMgOmega = 0.8f;  // damping of the phi-line block-Jacobi smoother
constexpr int kMgKLevels = 3;      // default: levels 1 .. kMgKLevels take K-cycle steps (when not the last)
constexpr int kMgKMax = 8;         // the deepest level a solve may ask K-cycle steps of

// The K-cycle depth a solve asks for: cycle 0 the default, 1 none (V-cycle), n >= 2
// levels 1 .. n.
int mg_kmax(const rt_solve_opts *o) { return o->cycle == 0 ? kMgKLevels : (o->cycle == 1 ? 0 : o->cycle); }

rt_status mg_prepare(rt_ctx *ctx)
{
    const Dims &d = ctx->d;
    RT_CHECK(ctx, d.n < (1L << 31), "multigrid: grids of 2^31 cells or more are not supported");
    if (!ctx->mg) {
        auto *h = new MgHier();
        h->nr = d.nr;
        std::vector<std::pair<int, int>> sh;
        mg_shapes(d.nt, d.np, sh);
        const int L = (int)sh.size() - 1;
        h->lev.resize(L + 1);
        bool ok = true;
        auto f32 = [&](long n) { float *p = dalloc<float>(ctx, n); ok = ok && p; return p; };
        auto f64 = [&](long n) { double *p = dalloc<double>(ctx, n); ok = ok && p; return p; };
        for (int l = 0; l <= L && ok; l++) {
            MgLevel &v = h->lev[l];
            v.nt = sh[l].first;
            v.np = sh[l].second;
            v.n = (long)d.nr * v.nt * v.np;
            const long lines = (long)d.nr * v.nt;
            if (l == 0) {
                v.dg = nullptr;
                v.ar = ctx->ahat32;
                v.at = ctx->ahat32 + d.n;
                v.ap = ctx->ahat32 + 2 * d.n;
            } else {
                h->d64.push_back(MgLevel64{f64(v.n), f64(v.n), f64(v.n), f64(v.n), f64(v.n)});
                h->dg32.push_back(f32(v.n));
                h->ar32.push_back(f32(v.n));
                h->at32.push_back(f32(v.n));
                h->ap32.push_back(f32(v.n));
                v.dg = h->dg32.back();
                v.ar = h->ar32.back();
                v.at = h->at32.back();
                v.ap = h->ap32.back();
            }
            if (l < L) {
                h->w.push_back(f32(v.n));
                h->im.push_back(f32(v.n));
                h->cp.push_back(f32(v.n));
                h->q.push_back(f32(v.n));
                h->g.push_back(f32(v.n));
                h->rho.push_back(f32(lines));
                h->kap.push_back(f32(lines));
                v.w = h->w.back();
                v.im = h->im.back();
                v.cp = h->cp.back();
                v.q = h->q.back();
                v.g = h->g.back();
                v.rho = h->rho.back();
                v.kap = h->kap.back();
                v.x = f32(v.n);
                v.dp = f32(v.n);
            }
            v.b = f32(v.n);
            v.x2 = f32(v.n);
            if (l > 0) v.xr = f32(v.n);
        }
        h->kl.resize(L + 1);
        for (int l = 1; l <= kMgKMax && l < L && ok; l++) {
            const long nl = h->lev[l].n;
            h->kl[l] = MgKLevel{f32(nl), f32(nl), f32(nl), f64(4)};
        }
        h->kpart = f64(8 * 4096);  // five sums for each of at most 4096 blocks
        h->B0 = f64(d.n);
        h->t64a = f64(d.n);
        h->t64b = f64(d.n);
        h->part = f64(2 * (long)((d.nr * (long)d.nt + 255) / 256));  // pairs, one per line-sweep block
        h->cnt = dalloc<unsigned>(ctx, 1);
        ok = ok && h->cnt;
        if (h->cnt && hipMemset(h->cnt, 0, sizeof(unsigned)) != hipSuccess) ok = false;
        h->cim = f64(d.nr);
        h->ccp = f64(d.nr);
        h->inv = f64((long)d.nr * d.nr);
        if (!ctx->mg_z) ctx->mg_z = f64(d.n);
        if (!ok) {
            delete h;
            return fail(ctx, RT_ENOMEM, "multigrid: out of device memory");
        }
        ctx->mg = h;
    }
    if (!ctx->mg->ready) {
        launch_mg_setup(*ctx->mg, ctx->ahat, ctx->s, ctx->stream);
        RT_HIP(ctx, hipGetLastError());
        ctx->mg->ready = true;
    }
    return RT_OK;
}

// Float64 flexible CG preconditioned by one multigrid cycle per iteration (float32 inside
// the cycle; the iteration's dots, vectors and the true residual stay float64).
rt_status solve_fp64_mg(rt_ctx *ctx, const rt_solve_opts *o, rt_solve_stats *st, double bb)
{
    const Dims &d = ctx->d;
    hipStream_t s = ctx->stream;
    DevScalars *h = ctx->h_sc;
    if (rt_status e = mg_prepare(ctx)) return e;
    MgHier &mg = *ctx->mg;
    mg.kmax = mg_kmax(o);
    h->thresh2 = o->tol * o->tol * bb;
    h->done = 0;
    h->iters = 0;
    h->beta = 0.0;
    if (rt_status e = write_scalars(ctx)) return e;
    launch_resid(d, ctx->nblk, ctx->ahat, ctx->bhat, ctx->y, ctx->r, ctx->partials, ctx->counter, ctx->sc, 1, s);
    if (rt_status e = read_scalars(ctx)) return e;
    double *pold = ctx->p0, *pnew = ctx->p1;
    const int every = o->check_every > 0 ? o->check_every : 8;
    rt_status status = RT_OK;
    double res = std::sqrt(h->res2 / bb);
    bool restart = true;
    for (;;) {
        st->relres = res;
        if (!isfin(res)) { status = RT_ENONFINITE; break; }
        if (res <= o->tol) break;
        if (h->iters >= o->max_iter) { status = RT_ENOCONV; break; }
        int m = std::min(every, o->max_iter - h->iters);
        int it_before = h->iters;
        for (int k = 0; k < m; k++) {
            const hipEvent_t *ev = k == 0 ? &ctx->ev[8] : nullptr;
            if (ev) (void)hipEventRecord(ev[0], s);
            launch_mg_vcycle(mg, ctx->r, ctx->mg_z, ctx->qv, kMgOmega, ctx->sc, restart && k == 0, s);
            if (ev) (void)hipEventRecord(ev[3], s);
            launch_pcg_dir_upd(d, ctx->nblk, ctx->nblk_upd, ctx->ahat, ctx->mg_z, ctx->y, ctx->r, pold, pnew, ctx->qv,
                               ctx->partials, ctx->counter, ctx->sc, s, ev);
            std::swap(pold, pnew);
        }
        restart = false;
        RT_HIP(ctx, hipGetLastError());
        if (rt_status e = read_scalars(ctx)) return e;
        add_kernel_sample(ctx, st, true);
        if ((h->iters - it_before) % 2 != m % 2) std::swap(pold, pnew);  // kernels that exited early
        if (!isfin(h->res2)) { status = RT_ENONFINITE; st->relres = NAN; break; }
        if (h->done || h->iters >= o->max_iter) {
            launch_resid(d, ctx->nblk, ctx->ahat, ctx->bhat, ctx->y, ctx->r, ctx->partials, ctx->counter,
                         ctx->sc, 1, s);
            if (rt_status e = read_scalars(ctx)) return e;
            res = std::sqrt(h->res2 / bb);
            restart = true;
        }
    }
    st->iters = h->iters;
    st->precond_applies = h->iters;
    return status;
}

// Flexible CG in float32 preconditioned by one V-cycle per iteration (the float32
// machinery of the learned mode: float64 dots, float64 reliable updates whenever r.r
// has fallen a hundredfold); a non-finite float32 state hands the solve to the float64
// multigrid CG from the last reliable iterate.
rt_status solve_mixed_mg(rt_ctx *ctx, const rt_solve_opts *o, rt_solve_stats *st, double bb)
{
    const Dims &d = ctx->d;
    hipStream_t s = ctx->stream;
    DevScalars *h = ctx->h_sc;
    if (rt_status e = mg_prepare(ctx)) return e;
    MgHier &mg = *ctx->mg;
    mg.kmax = mg_kmax(o);
    const double delta2 = 0.01;
    h->iters = 0;
    h->done = 0;
    h->beta = 0.0;
    h->thresh2 = o->tol * o->tol * bb;
    if (rt_status e = write_scalars(ctx)) return e;
    launch_resid(d, ctx->nblk, ctx->ahat, ctx->bhat, ctx->y, ctx->r, ctx->partials, ctx->counter, ctx->sc, 0, s);
    launch_reliable(d, ctx->nblk, ctx->r, ctx->r32, ctx->x32, ctx->partials, ctx->counter, ctx->sc, 1, s);
    if (rt_status e = read_scalars(ctx)) return e;
    double res = std::sqrt(h->res2 / bb), rr_ref = h->res2;
    float *pold = ctx->p32a, *pnew = ctx->p32b;
    rt_status status = RT_OK;
    bool nonfinite = false;
    int applies = 0;
    for (;;) {
        st->relres = res;
        if (!isfin(res)) { nonfinite = true; break; }
        if (res <= o->tol) break;
        if (h->iters >= o->max_iter) { status = RT_ENOCONV; break; }
        const bool sample = applies % 8 == 0;
        if (sample) (void)hipEventRecord(ctx->ev[8], s);
        launch_mg_vcycle32(mg, ctx->r32, ctx->z32, kMgOmega, ctx->sc, s);
        applies++;
        if (applies > 1) launch_fcg_beta(d, ctx->nblk, ctx->z32, ctx->q32, ctx->partials, ctx->counter, ctx->sc, s);
        if (sample) (void)hipEventRecord(ctx->ev[11], s);
        launch_fcg_dir(d, ctx->nblk, ctx->ahat32, ctx->z32, pold, ctx->r32, pnew, ctx->q32, ctx->partials,
                       ctx->counter, ctx->sc, s);
        if (sample) (void)hipEventRecord(ctx->ev[9], s);
        launch_cg_upd32(d, ctx->nblk_upd, ctx->x32, pnew, ctx->r32, ctx->q32, ctx->partials, ctx->counter, ctx->sc, s);
        if (sample) (void)hipEventRecord(ctx->ev[10], s);
        std::swap(pold, pnew);
        RT_HIP(ctx, hipGetLastError());
        if (rt_status e = read_scalars(ctx)) return e;
        if (sample) add_kernel_sample(ctx, st, true);
        if (!isfin(h->rr) || !isfin(h->alpha)) { nonfinite = true; break; }
        if (h->done || h->rr <= delta2 * rr_ref || h->iters >= o->max_iter) {
            launch_fold(d.n, ctx->x32, ctx->y, s);
            launch_resid(d, ctx->nblk, ctx->ahat, ctx->bhat, ctx->y, ctx->r, ctx->partials, ctx->counter,
                         ctx->sc, 0, s);
            launch_reliable(d, ctx->nblk, ctx->r, ctx->r32, ctx->x32, ctx->partials, ctx->counter, ctx->sc, 0, s);
            RT_HIP(ctx, hipGetLastError());
            if (rt_status e = read_scalars(ctx)) return e;
            res = std::sqrt(h->res2 / bb);
            rr_ref = h->res2;
            st->outer_iters++;
        }
    }
    st->iters = h->iters;
    st->precond_applies = applies;
    if (nonfinite) {
        if (rt_status e = reset_directions(ctx)) return e;
        st->fallback = 1;
        rt_solve_stats s64{};
        rt_solve_opts o64 = *o;
        o64.mode = RT_SOLVE_FP64;
        o64.max_iter = std::max(1, o->max_iter - st->iters);
        status = solve_fp64_mg(ctx, &o64, &s64, bb);
        st->iters += s64.iters;
        st->precond_applies += s64.precond_applies;
        st->relres = s64.relres;
    }
    return status;
}

rt_status solve_gmres(rt_ctx *ctx, const rt_solve_opts *o, rt_solve_stats *st, double bb, rt_net *net = nullptr,
                      int budget = 0, int *out = nullptr);

// Learned mode: flexible CG (Notay's FCG with one A-orthogonalisation, since the
// network is a nonlinear preconditioner) in float32 with float64 dots and the same
// float64 reliable updates as the mixed mode; z = M(r) is the U-Net applied to the
// residual scaled to unit RMS.  If the true residual is not below tol after
// inner_max_iter network applications (default 400), or anything turns non-finite,
// the solve falls back to float64 CG from the current iterate.
rt_status solve_learned(rt_ctx *ctx, const rt_solve_opts *o, rt_solve_stats *st, double bb, bool allow_fallback = true)
{
    const Dims &d = ctx->d;
    hipStream_t s = ctx->stream;
    DevScalars *h = ctx->h_sc;
    rt_net *net = o->net;
    const double delta2 = 0.01;
    const int budget = o->inner_max_iter > 0 ? o->inner_max_iter : 400;
    if (rt_status e = net_prepare(net, ctx)) return fail(ctx, e, std::string("network: ") + rt_net_last_error(net));
    rt_status status = RT_OK;
    bool fallback = false, nonfinite = false;
    const bool fgmres = o->inner == RT_INNER_FGMRES;
    if (fgmres) {
        // flexible GMRES(m) in float64 with the network as the right preconditioner; it
        // updates y itself, so there is no float32 iterate to fold in afterwards
        int out = 0;
        status = solve_gmres(ctx, o, st, bb, net, budget, &out);
        if (status == RT_ENONFINITE) {
            status = RT_OK;
            fallback = nonfinite = true;
        } else if (status == RT_OK && out == 1) {
            fallback = true;
        }
        if (status != RT_OK || !fallback) return status;
    } else {
    h->iters = 0;
    h->done = 0;
    h->beta = 0.0;
    h->thresh2 = o->tol * o->tol * bb;
    if (rt_status e = write_scalars(ctx)) return e;
    launch_resid(d, ctx->nblk, ctx->ahat, ctx->bhat, ctx->y, ctx->r, ctx->partials, ctx->counter, ctx->sc, 0, s);
    launch_reliable(d, ctx->nblk, ctx->r, ctx->r32, ctx->x32, ctx->partials, ctx->counter, ctx->sc, 1, s);
    if (rt_status e = read_scalars(ctx)) return e;
    double res = std::sqrt(h->res2 / bb), rr_ref = h->res2;
    float *pold = ctx->p32a, *pnew = ctx->p32b;
    for (;;) {
        st->relres = res;
        if (!isfin(res)) { fallback = nonfinite = true; break; }
        if (res <= o->tol) break;
        if (h->iters >= o->max_iter) { status = RT_ENOCONV; break; }
        if (st->precond_applies >= budget) { fallback = true; break; }
        // z = M(r); p = z + beta p_old, q = A p, alpha; x, r update; beta for the next step
        if (rt_status e = net_precond(net, ctx, ctx->r32, ctx->z32))
            return fail(ctx, e, std::string("network: ") + rt_net_last_error(net));
        st->precond_applies++;
        if (st->precond_applies > 1)
            launch_fcg_beta(d, ctx->nblk, ctx->z32, ctx->q32, ctx->partials, ctx->counter, ctx->sc, s);
        launch_fcg_dir(d, ctx->nblk, ctx->ahat32, ctx->z32, pold, ctx->r32, pnew, ctx->q32, ctx->partials,
                       ctx->counter, ctx->sc, s);
        launch_cg_upd32(d, ctx->nblk_upd, ctx->x32, pnew, ctx->r32, ctx->q32, ctx->partials, ctx->counter, ctx->sc, s);
        std::swap(pold, pnew);
        RT_HIP(ctx, hipGetLastError());
        if (rt_status e = read_scalars(ctx)) return e;
        if (!isfin(h->rr) || !isfin(h->alpha)) { fallback = nonfinite = true; break; }
        if (h->done || h->rr <= delta2 * rr_ref || h->iters >= o->max_iter) {
            launch_fold(d.n, ctx->x32, ctx->y, s);
            launch_resid(d, ctx->nblk, ctx->ahat, ctx->bhat, ctx->y, ctx->r, ctx->partials, ctx->counter,
                         ctx->sc, 0, s);
            launch_reliable(d, ctx->nblk, ctx->r, ctx->r32, ctx->x32, ctx->partials, ctx->counter, ctx->sc, 0, s);
            RT_HIP(ctx, hipGetLastError());
            if (rt_status e = read_scalars(ctx)) return e;
            res = std::sqrt(h->res2 / bb);
            rr_ref = h->res2;
            st->outer_iters++;
        }
    }
    st->iters = h->iters;
    }
    if (fallback && !allow_fallback) {
        if (!nonfinite && !fgmres) launch_fold(d.n, ctx->x32, ctx->y, s);
        RT_HIP(ctx, hipGetLastError());
        return nonfinite ? RT_ENONFINITE : RT_OK;
    }
    if (fallback) {
        // keep what the float32 iterations gained (unless they went non-finite: then y is
        // the iterate of the last reliable update, and the direction buffers the network's
        // output reached are cleared), then finish with the float64 method.  Running out
        // of network applications is the planned hand-over (`handover`); `fallback`
        // marks a network that failed (non-finite output).
        if (!nonfinite) {
            if (!fgmres) launch_fold(d.n, ctx->x32, ctx->y, s);
        } else if (rt_status e = reset_directions(ctx)) {
            return e;
        }
        if (nonfinite) st->fallback = 1;
        else st->handover = 1;
        rt_solve_stats s64{};
        rt_solve_opts o64 = *o;
        o64.max_iter = std::max(1, o->max_iter - st->iters);
        if (o->reduce && rb_possible(ctx)) {
            // finish with the reduced mixed solve (its own guards hand over to reduced float64)
            o64.mode = RT_SOLVE_MIXED;
            status = solve_mixed_rb(ctx, &o64, &s64, bb);
            st->reduced = 1;
            st->outer_iters += s64.outer_iters;
        } else {
            o64.mode = RT_SOLVE_FP64;
            status = solve_fp64(ctx, &o64, &s64, bb);
        }
        st->iters += s64.iters;
        st->relres = s64.relres;
        st->ms_dir = s64.ms_dir;
        st->ms_upd = s64.ms_upd;
        st->ms_black = s64.ms_black;
        st->kernel_samples = s64.kernel_samples;
    }
    return status;
}

// Restarted GMRES(m) on A^ in float64 (the paper's solver class).  Arnoldi with
// classical Gram-Schmidt applied twice (CGS2: the projections of each pass are one
// deterministic batched reduction over the basis), Givens rotations of the Hessenberg
// column on the host, |g_(j+1)| as the residual estimate; a cycle ends after m steps
// or at the estimate tol, then y += V z (H z = g) and the true residual decides.
//
// With a network (flexible GMRES, Saad's FGMRES(m): right preconditioning by an
// operator that may change from step to step): step j applies the network to v_j
// (rounded to float32, scaled to unit RMS inside the application) and keeps the answer
// z_j in a second basis Z; w = A^ z_j enters the Arnoldi process, and the cycle's update
// is y += Z z, so |g_(j+1)| estimates the true residual of that update.  At most
// `budget` network applications: when they run out the cycle is closed with the steps
// taken (*out = 1); a non-finite network output ends the solve before it reaches y
// (*out = 2, y keeps the previous cycle's iterate).
rt_status solve_gmres(rt_ctx *ctx, const rt_solve_opts *o, rt_solve_stats *st, double bb, rt_net *net, int budget,
                      int *out)
{
    const Dims &d = ctx->d;
    const long n = d.n;
    hipStream_t s = ctx->stream;
    DevScalars *h = ctx->h_sc;
    const int m = o->restart > 0 ? o->restart : 30;
    if (m + 1 > kMaxBasis) return fail(ctx, RT_EINVAL, "restart must be at most 63");
    if (ctx->gm_cap < m + 1) {
        ctx->gmV = dalloc<double>(ctx, (size_t)(m + 1) * n);
        if (!ctx->gmV) return fail(ctx, RT_ENOMEM, "GMRES basis: out of device memory");
        ctx->gm_cap = m + 1;
        if (!ctx->gm_part) {
            ctx->gm_part = dalloc<double>(ctx, (size_t)ctx->nblk * kMaxBasis);
            ctx->gm_coef = dalloc<double>(ctx, kMaxBasis);
            if (!ctx->gm_part || !ctx->gm_coef) return fail(ctx, RT_ENOMEM, "GMRES workspace: out of device memory");
        }
    }
    if (net && ctx->gmz_cap < m) {
        ctx->gmZ = dalloc<double>(ctx, (size_t)m * n);
        if (!ctx->gmZ) return fail(ctx, RT_ENOMEM, "flexible GMRES basis: out of device memory");
        ctx->gmz_cap = m;
    }
    if (out) *out = 0;
    double *V = ctx->gmV;
    double *Z = net ? ctx->gmZ : ctx->gmV;  // the vectors the update combines
    const double bn = std::sqrt(bb);
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1), hc(kMaxBasis), h2(kMaxBasis);
    auto col = [&](int i, int j) -> double & { return H[(size_t)i * m + j]; };
    h->thresh2 = 0.0;
    if (rt_status e = write_scalars(ctx)) return e;
    rt_status status = RT_OK;
    int it = 0;
    bool spent = false;
    for (;;) {
        // r0 = b - A y, its norm; v_0 = r0 / beta
        launch_resid(d, ctx->nblk, ctx->ahat, ctx->bhat, ctx->y, ctx->r, ctx->partials, ctx->counter, ctx->sc, 0, s);
        RT_HIP(ctx, hipGetLastError());
        if (rt_status e = read_scalars(ctx)) return e;
        const double beta = std::sqrt(h->res2);
        st->relres = beta / bn;
        if (!isfin(beta)) { status = RT_ENONFINITE; break; }
        if (st->relres <= o->tol) break;
        if (it >= o->max_iter) { status = RT_ENOCONV; break; }
        if (spent) { if (out) *out = 1; break; }
        launch_scale_into(n, ctx->r, 1.0 / beta, V, s);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m && it < o->max_iter; j++) {
            if (net && st->precond_applies >= budget) { spent = true; break; }
            it++;
            double *w = V + (size_t)(j + 1) * n;
            const double *src = V + (size_t)j * n;
            if (net) {  // z_j = M(v_j)
                launch_d2f(n, src, ctx->r32, s);
                launch_norm2_rr32(d, ctx->nblk, ctx->r32, ctx->partials, ctx->counter, ctx->sc, s);
                if (rt_status e = net_precond(net, ctx, ctx->r32, ctx->z32))
                    return fail(ctx, e, std::string("network: ") + rt_net_last_error(net));
                st->precond_applies++;
                launch_f2d(n, ctx->z32, Z + (size_t)j * n, s);
                src = Z + (size_t)j * n;
            }
            launch_spmv(d, ctx->nblk, ctx->ahat, src, w, s);
            for (int pass = 0; pass < 2; pass++) {  // CGS2
                launch_mdot(d, ctx->nblk, V, j + 1, w, ctx->gm_part, ctx->gm_coef, s);
                RT_HIP(ctx, hipMemcpyAsync(pass ? h2.data() : hc.data(), ctx->gm_coef, (j + 1) * sizeof(double),
                                           hipMemcpyDeviceToHost, s));
                launch_maxpy(n, V, j + 1, ctx->gm_coef, -1.0, w, s);
            }
            launch_norm2(d, ctx->nblk, w, ctx->partials, ctx->counter, ctx->sc, s);
            RT_HIP(ctx, hipGetLastError());
            if (rt_status e = read_scalars(ctx)) return e;  // also completes the two copies above
            const double hn = std::sqrt(h->res2);
            bool fin = isfin(hn);
            for (int i = 0; i <= j; i++) fin = fin && isfin(hc[i] + h2[i]);
            if (!fin) {
                status = RT_ENONFINITE;
                if (net && out) *out = 2;
                break;
            }
            for (int i = 0; i <= j; i++) col(i, j) = hc[i] + h2[i];
            col(j + 1, j) = hn;
            if (hn > 0.0) launch_scale_into(n, w, 1.0 / hn, w, s);
            for (int i = 0; i < j; i++) {
                const double a = col(i, j), b = col(i + 1, j);
                col(i, j) = cs[i] * a + sn[i] * b;
                col(i + 1, j) = -sn[i] * a + cs[i] * b;
            }
            const double a = col(j, j), b = col(j + 1, j);
            const double dd = std::sqrt(a * a + b * b);
            cs[j] = dd > 0.0 ? a / dd : 1.0;
            sn[j] = dd > 0.0 ? b / dd : 0.0;
            col(j, j) = dd;
            col(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            k = j + 1;
            if (std::fabs(g[j + 1]) / bn <= o->tol || hn == 0.0) break;
        }
        if (status != RT_OK) break;
        if (k == 0) {  // no step taken: the network budget is spent (or the iteration
            if (spent) {  // limit reached, which the next pass reports)
                if (out) *out = 1;
                break;
            }
            continue;
        }
        for (int i = k - 1; i >= 0; i--) {  // H_k z = g_k
            double t = g[i];
            for (int l = i + 1; l < k; l++) t -= col(i, l) * g[l];
            g[i] = t / col(i, i);
        }
        RT_HIP(ctx, hipMemcpyAsync(ctx->gm_coef, g.data(), k * sizeof(double), hipMemcpyHostToDevice, s));
        launch_maxpy(n, Z, k, ctx->gm_coef, 1.0, ctx->y, s);
        RT_HIP(ctx, hipStreamSynchronize(s));  // g is reused by the next cycle
        st->outer_iters++;
    }
    st->iters = it;
    return status;
}

}  // namespace

extern "C" {

rt_status rt_fld_solve(rt_ctx *ctx, const rt_solve_opts *o, double *E, rt_solve_stats *st)
{
    if (!ctx) return fail(nullptr, RT_EINVAL, "context is NULL");
    RT_CHECK(ctx, ctx->have_system, "no assembled system");
    RT_CHECK(ctx, o && E, "rt_fld_solve: NULL argument");
    if (o->mode == RT_SOLVE_NONE) {  // no transport: the background field of the boundary
        if (st) *st = rt_solve_stats{};
        launch_fill(ctx->d.n, ctx->Eb, E, ctx->stream);
        RT_HIP(ctx, hipGetLastError());
        return RT_OK;
    }
    RT_CHECK(ctx, o->tol > 0.0 && o->tol < 1.0, "tol must be in (0, 1)");
    RT_CHECK(ctx, o->max_iter > 0, "max_iter must be positive");
    RT_CHECK(ctx, o->mode == RT_SOLVE_FP64 || o->mode == RT_SOLVE_MIXED || o->mode == RT_SOLVE_LEARNED ||
                      o->mode == RT_SOLVE_GMRES,
             "unknown solve mode");
    RT_CHECK(ctx, o->mode != RT_SOLVE_LEARNED || o->net, "learned mode needs a network");
    RT_CHECK(ctx, o->inner == RT_INNER_FCG || o->inner == RT_INNER_FGMRES, "inner must be an rt_inner value");
    RT_CHECK(ctx, o->cycle >= 0 && o->cycle <= kMgKMax,
             "cycle must be 0 (K-cycle steps on levels 1-3), 1 (V-cycle) or 2..8 (K-cycle steps on levels 1..cycle)");
    RT_CHECK(ctx, o->launch >= RT_LAUNCH_AUTO && o->launch <= RT_LAUNCH_BLOCK,
             "rt_fld_solve: launch must be an rt_launch value");
    RT_CHECK(ctx, o->precond == 0 || (o->precond == 1 && o->mode == RT_SOLVE_FP64 && !o->reduce) ||
                      (o->precond == 2 && (o->mode == RT_SOLVE_FP64 || o->mode == RT_SOLVE_MIXED) && !o->reduce),
             "precond = 1 (radial-line block Jacobi) needs RT_SOLVE_FP64, precond = 2 (multigrid) RT_SOLVE_FP64 "
             "or RT_SOLVE_MIXED, both without reduce");
    rt_solve_stats local{};
    rt_solve_stats *S = st ? st : &local;
    *S = rt_solve_stats{};
    Clock clk;
    double bb = 0.0;
    if (rt_status e = norm_b(ctx, bb)) return e;
    if (!isfin(bb)) {
        S->status = RT_ENONFINITE;
        return fail(ctx, RT_ENONFINITE, "right-hand side is not finite");
    }
    if (bb == 0.0) bb = 1.0;
    launch_scale_div(ctx->d.n, ctx->s, E, ctx->y, ctx->stream);  // y0 = E / s
    rt_status status;
    const bool rb = o->reduce && rb_possible(ctx);
    if (o->mode == RT_SOLVE_FP64 && o->precond == 1) status = solve_fp64_line(ctx, o, S, bb);
    else if (o->mode == RT_SOLVE_FP64 && o->precond == 2) status = solve_fp64_mg(ctx, o, S, bb);
    else if (o->mode == RT_SOLVE_MIXED && o->precond == 2) status = solve_mixed_mg(ctx, o, S, bb);
    else if (o->mode == RT_SOLVE_FP64) status = rb ? solve_fp64_rb(ctx, o, S, bb) : solve_fp64(ctx, o, S, bb);
    else if (o->mode == RT_SOLVE_MIXED) status = rb ? solve_mixed_rb(ctx, o, S, bb) : solve_mixed(ctx, o, S, bb);
    else if (o->mode == RT_SOLVE_GMRES) status = solve_gmres(ctx, o, S, bb);
    else status = solve_learned(ctx, o, S, bb);
    if (status == RT_EDEVICE) return status;
    launch_scale_mul(ctx->d.n, ctx->s, ctx->y, E, ctx->stream);  // E = s y
    RT_HIP(ctx, hipGetLastError());
    RT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    S->status = status;
    S->ms = clk.ms();
    if (status == RT_ENOCONV) return fail(ctx, status, "iteration limit reached");
    if (status == RT_ENONFINITE) {
        if (rt_status e = reset_directions(ctx)) return e;
        return fail(ctx, status, "non-finite residual");
    }
    return status;
}

}  // extern "C"

namespace rt {
// `applies` iterations of the learned flexible CG from y (device, y-space, in/out), with
// no float64 fallback (training-data generation: the residuals the learned solver
// itself meets).  Stops early at the relative residual 1e-12.
rt_status learned_from(rt_ctx *ctx, rt_net *net, int applies, double *y, rt_solve_stats *st)
{
    if (!ctx->have_system) return fail(ctx, RT_EINVAL, "no assembled system");
    rt_solve_stats local{};
    rt_solve_stats *S = st ? st : &local;
    *S = rt_solve_stats{};
    double bb = 0.0;
    if (rt_status e = norm_b(ctx, bb)) return e;
    if (!(bb > 0.0) || !isfin(bb)) return fail(ctx, RT_ENONFINITE, "right-hand side is zero or not finite");
    RT_HIP(ctx, hipMemcpyAsync(ctx->y, y, ctx->d.n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    rt_solve_opts o{};
    o.mode = RT_SOLVE_LEARNED;
    o.tol = 1e-12;
    o.max_iter = applies;
    o.inner_max_iter = applies;
    o.net = net;
    rt_status status = applies > 0 ? solve_learned(ctx, &o, S, bb, false) : RT_OK;
    RT_HIP(ctx, hipMemcpyAsync(y, ctx->y, ctx->d.n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    RT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return status == RT_ENOCONV ? RT_OK : status;
}

rt_status solve_fp64_from(rt_ctx *ctx, double tol, int max_iter, double *y, rt_solve_stats *st)
{
    if (!ctx->have_system) return fail(ctx, RT_EINVAL, "no assembled system");
    rt_solve_stats local{};
    rt_solve_stats *S = st ? st : &local;
    *S = rt_solve_stats{};
    double bb = 0.0;
    if (rt_status e = norm_b(ctx, bb)) return e;
    if (!(bb > 0.0) || !isfin(bb)) return fail(ctx, RT_ENONFINITE, "right-hand side is zero or not finite");
    RT_HIP(ctx, hipMemcpyAsync(ctx->y, y, ctx->d.n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    rt_solve_opts o{};
    o.mode = RT_SOLVE_FP64;
    o.tol = tol;
    o.max_iter = max_iter;
    o.check_every = std::min(32, max_iter);
    rt_status status = solve_fp64(ctx, &o, S, bb);
    RT_HIP(ctx, hipMemcpyAsync(y, ctx->y, ctx->d.n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    RT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return status == RT_ENOCONV ? RT_OK : status;
}

// ------------------------------------------------------------- step graph
//
// A main-loop step whose solve is the reduced float64 CG in one workgroup (or that runs
// without transport) is a fixed sequence of launches once the solver's host set-up (the
// stopping threshold from ||b^||^2, read back) moves to the device: rt_relax captures it
// in one HIP graph and replays the graph every step, reading the scalars back once.  The
// launches are those of rt_step with that solve, in the same order and with the same
// arguments, except that the host's loop over chunks of iterations becomes one block
// launch followed by the true residual; where the host-driven loop would have decided
// otherwise (a non-finite value, a chunk used up, a true residual above tol) the step is
// redone on that path from the saved temperature, so the results are the same bits.
bool step_graph_applies(const rt_ctx *ctx, const rt_solve_opts *o)
{
    if (o->launch != RT_LAUNCH_AUTO) return false;
    if (o->mode == RT_SOLVE_NONE) return true;
    return o->mode == RT_SOLVE_FP64 && o->reduce && o->precond == 0 && o->tol > 0.0 && o->tol < 1.0 &&
           o->max_iter > 0 && rb_possible(ctx) && use_block(o, rb_half(ctx->d));
}

int step_graph_chunk(const rt_solve_opts *o) { return std::min(kBlockChunk, o->max_iter); }

// The step's launches on ctx->stream (T^n saved to ctx->Tn, the change written to the
// scalars); no host synchronisation.
rt_status enqueue_step(rt_ctx *ctx, const rt_fld_params *p, const rt_solve_opts *o, const double *rho, double *T,
                       double *E)
{
    const long n = ctx->d.n;
    hipStream_t s = ctx->stream;
    RT_HIP(ctx, hipMemcpyAsync(ctx->Tn, T, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (rt_status e = rt_raytrace(ctx, nullptr, nullptr, rho, T, ctx->q, ctx->S, nullptr, nullptr)) return e;
    if (rt_status e = rt_energy(ctx, nullptr, p, T, ctx->S, ctx->En)) return e;
    if (rt_status e = rt_fld_assemble(ctx, nullptr, p, rho, T, ctx->En, ctx->q, nullptr, nullptr)) return e;
    if (o->mode == RT_SOLVE_NONE) {
        launch_fill(n, ctx->Eb, E, s);
    } else {
        RT_HIP(ctx, hipMemcpyAsync(E, ctx->En, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        launch_norm2(ctx->d, ctx->nblk, ctx->bhat, ctx->partials, ctx->counter, ctx->sc, s);
        launch_solve_init(ctx->sc, o->tol * o->tol, s);
        launch_scale_div(n, ctx->s, E, ctx->y, s);  // y0 = E / s
        // the buffers of solve_fp64_rb
        const Dims dh = rb_half(ctx->d);
        const long nh = dh.n;
        double *rb = ctx->r, *tr = ctx->r + nh, *pold = ctx->p0, *yb = ctx->qv + nh, *rhs = ctx->p1;
        if (rt_status e = rb_prepare(ctx, rhs, yb, rb)) return e;
        rb_resid(ctx, rhs, yb, rb, tr, 1);
        if (!launch_rb_cg_block(dh, ctx->rb_a, yb, rb, pold, step_graph_chunk(o), ctx->sc, s))
            return fail(ctx, RT_EDEVICE, "one-workgroup CG: grid too large");
        rb_resid(ctx, rhs, yb, rb, tr, 1);
        if (rt_status e = rb_finish(ctx, rhs, yb, tr)) return e;
        launch_scale_mul(n, ctx->s, ctx->y, E, s);  // E = s y
    }
    launch_newton(ctx->d, ctx->op, E, ctx->S, T, s);
    double *dchange = reinterpret_cast<double *>(reinterpret_cast<char *>(ctx->sc) + offsetof(DevScalars, change));
    launch_max_change(n, ctx->nblk, T, ctx->Tn, ctx->partials, ctx->counter, dchange, s);
    RT_HIP(ctx, hipGetLastError());
    return RT_OK;
}

// Captures enqueue_step on the context's capture stream (ctx->stream may be the legacy
// default stream, which cannot be captured) and instantiates it.
rt_status capture_step(rt_ctx *ctx, const rt_fld_params *p, const rt_solve_opts *o, const double *rho, double *T,
                       double *E, hipGraphExec_t *ex)
{
    *ex = nullptr;
    if (o->mode != RT_SOLVE_NONE && !ctx->rb_a) {  // rb_prepare's allocation, made before capturing
        ctx->rb_a = dalloc<double>(ctx, 3 * ctx->d.n);
        ctx->rb_a32 = dalloc<float>(ctx, 3 * ctx->d.n);
        if (!ctx->rb_a || !ctx->rb_a32) return fail(ctx, RT_ENOMEM, "red-black split: out of device memory");
    }
    if (!ctx->cap_stream) RT_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    const hipStream_t saved = ctx->stream;
    RT_HIP(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    ctx->stream = ctx->cap_stream;
    const rt_status e = enqueue_step(ctx, p, o, rho, T, E);
    ctx->stream = saved;
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &g);
    if (e != RT_OK) {
        if (g) (void)hipGraphDestroy(g);
        return e;
    }
    if (ec != hipSuccess || !g) return fail(ctx, RT_EDEVICE, std::string("step capture: ") + hipGetErrorString(ec));
    const hipError_t ei = hipGraphInstantiate(ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(ctx, RT_EDEVICE, std::string("step graph instantiation: ") + hipGetErrorString(ei));
    return RT_OK;
}

// Whether the host-driven step would have ended as the replay did (scalars read back).
bool step_graph_result_ok(const DevScalars *h, const rt_solve_opts *o)
{
    if (!isfin(h->change)) return false;
    if (o->mode == RT_SOLVE_NONE) return true;
    if (!isfin(h->bnorm2) || !isfin(h->rr) || !isfin(h->res2)) return false;
    const double res = std::sqrt(h->res2 / h->bnorm2);
    return h->iters < step_graph_chunk(o) && h->done && res <= o->tol;
}
}  // namespace rt

extern "C" {

rt_status rt_temperature(rt_ctx *ctx, const rt_opacity *op, const double *E, const double *S_abs, double *T)
{
    if (!ctx) return fail(nullptr, RT_EINVAL, "context is NULL");
    if (op) { rt_status s = rt_set_opacity(ctx, op); if (s) return s; }
    RT_CHECK(ctx, ctx->have_opac, "no opacity table on the context");
    RT_CHECK(ctx, E && S_abs && T, "rt_temperature: NULL field pointer");
    launch_newton(ctx->d, ctx->op, E, S_abs, T, ctx->stream);
    RT_HIP(ctx, hipGetLastError());
    return RT_OK;
}

rt_status rt_force(rt_ctx *ctx, const double *E, const double *q_star, double *f)
{
    if (!ctx) return fail(nullptr, RT_EINVAL, "context is NULL");
    RT_CHECK(ctx, ctx->have_system, "no assembled system");
    RT_CHECK(ctx, E && q_star && f, "rt_force: NULL field pointer");
    launch_force(ctx->d, ctx->geo, ctx->w, ctx->chi, E, q_star, ctx->Eb, f, ctx->stream);
    RT_HIP(ctx, hipGetLastError());
    return RT_OK;
}

rt_status rt_step(rt_ctx *ctx, const rt_opacity *op, const rt_star *st, const rt_fld_params *p,
                  const rt_solve_opts *o, const double *rho, double *T, double *E, double *f_rad,
                  rt_step_stats *stats)
{
    if (!ctx) return fail(nullptr, RT_EINVAL, "context is NULL");
    RT_CHECK(ctx, rho && T && E && o, "rt_step: NULL argument");
    if (rt_status s = check_fld(ctx, p)) return s;
    hipStream_t s = ctx->stream;
    Clock clk;
    RT_HIP(ctx, hipEventRecord(ctx->ev[0], s));
    if (rt_status e = rt_raytrace(ctx, op, st, rho, T, ctx->q, ctx->S, nullptr, nullptr)) return e;
    RT_HIP(ctx, hipEventRecord(ctx->ev[1], s));
    if (rt_status e = rt_energy(ctx, nullptr, p, T, ctx->S, ctx->En)) return e;
    if (rt_status e = rt_fld_assemble(ctx, nullptr, p, rho, T, ctx->En, ctx->q, nullptr, nullptr)) return e;
    RT_HIP(ctx, hipMemcpyAsync(E, ctx->En, ctx->d.n * sizeof(double), hipMemcpyDeviceToDevice, s));
    RT_HIP(ctx, hipEventRecord(ctx->ev[2], s));
    rt_solve_stats sst{};
    rt_status solve_status = rt_fld_solve(ctx, o, E, &sst);
    if (solve_status != RT_OK && solve_status != RT_ENOCONV) return solve_status;
    RT_HIP(ctx, hipEventRecord(ctx->ev[3], s));
    if (rt_status e = rt_temperature(ctx, nullptr, E, ctx->S, T)) return e;
    RT_HIP(ctx, hipEventRecord(ctx->ev[4], s));
    if (f_rad)
        if (rt_status e = rt_force(ctx, E, ctx->q, f_rad)) return e;
    RT_HIP(ctx, hipEventRecord(ctx->ev[5], s));
    if (stats) {
        RT_HIP(ctx, hipEventSynchronize(ctx->ev[5]));
        float t01, t12, t23, t34, t05;
        RT_HIP(ctx, hipEventElapsedTime(&t01, ctx->ev[0], ctx->ev[1]));
        RT_HIP(ctx, hipEventElapsedTime(&t12, ctx->ev[1], ctx->ev[2]));
        RT_HIP(ctx, hipEventElapsedTime(&t23, ctx->ev[2], ctx->ev[3]));
        RT_HIP(ctx, hipEventElapsedTime(&t34, ctx->ev[3], ctx->ev[4]));
        RT_HIP(ctx, hipEventElapsedTime(&t05, ctx->ev[0], ctx->ev[5]));
        stats->solve = sst;
        stats->ms_raytrace = t01;
        stats->ms_assemble = t12;
        stats->ms_solve = t23;
        stats->ms_newton = t34;
        stats->ms_total = t05;
        (void)clk;
    }
    if (solve_status == RT_ENOCONV) return fail(ctx, RT_ENOCONV, "iteration limit reached");
    return RT_OK;
}

rt_status rt_step_fields(rt_ctx *ctx, const double **q_star, const double **S_abs, const double **E_n)
{
    if (!ctx) return fail(nullptr, RT_EINVAL, "context is NULL");
    if (q_star) *q_star = ctx->q;
    if (S_abs) *S_abs = ctx->S;
    if (E_n) *E_n = ctx->En;
    return RT_OK;
}

rt_status rt_precond_apply(rt_ctx *ctx, const double *r, double *z)
{
    if (!ctx) return fail(nullptr, RT_EINVAL, "context is NULL");
    RT_CHECK(ctx, ctx->have_system, "no assembled system");
    RT_CHECK(ctx, r && z, "rt_precond_apply: NULL field pointer");
    const long n = ctx->d.n;
    if (!ctx->ln_c) {
        ctx->ln_c = dalloc<double>(ctx, n);
        ctx->ln_im = dalloc<double>(ctx, n);
        ctx->ln_z = dalloc<double>(ctx, n);
        if (!ctx->ln_c || !ctx->ln_im || !ctx->ln_z) return fail(ctx, RT_ENOMEM, "line preconditioner: out of device memory");
    }
    if (!ctx->ln_ready) {
        launch_line_factor(ctx->d, ctx->nblk, ctx->ahat, ctx->ln_c, ctx->ln_im, ctx->stream);
        ctx->ln_ready = true;
    }
    ctx->h_sc->done = 0;
    ctx->h_sc->rr = 0.0;
    if (rt_status e = write_scalars(ctx)) return e;
    launch_line_solve(ctx->d, ctx->nblk, ctx->ahat, ctx->ln_c, ctx->ln_im, r, z, ctx->partials, ctx->counter, ctx->sc,
                      1, ctx->stream);
    RT_HIP(ctx, hipGetLastError());
    return RT_OK;
}

rt_status rt_mg_apply(rt_ctx *ctx, const double *r, double *z)
{
    if (!ctx) return fail(nullptr, RT_EINVAL, "context is NULL");
    RT_CHECK(ctx, ctx->have_system, "no assembled system");
    RT_CHECK(ctx, r && z, "rt_mg_apply: NULL field pointer");
    if (rt_status e = mg_prepare(ctx)) return e;
    // the solver's own cycle (its r.z and scalars land in the context's scalars)
    ctx->mg->kmax = kMgKLevels;
    ctx->h_sc->done = 0;
    ctx->h_sc->rr = 0.0;
    if (rt_status e = write_scalars(ctx)) return e;
    launch_mg_vcycle(*ctx->mg, r, z, ctx->qv, kMgOmega, ctx->sc, 1, ctx->stream);
    RT_HIP(ctx, hipGetLastError());
    return RT_OK;
}

rt_status rt_mg_level(rt_ctx *ctx, int level, rt_mg_level_view *out)
{
    if (!ctx) return fail(nullptr, RT_EINVAL, "context is NULL");
    RT_CHECK(ctx, ctx->have_system, "no assembled system");
    RT_CHECK(ctx, out, "rt_mg_level: NULL view");
    if (rt_status e = mg_prepare(ctx)) return e;
    const MgHier &mg = *ctx->mg;
    const int L = (int)mg.lev.size() - 1;
    RT_CHECK(ctx, level >= 0 && level <= L, "rt_mg_level: level out of range");
    const MgLevel &v = mg.lev[level];
    *out = rt_mg_level_view{};
    out->levels = L + 1;
    out->nr = ctx->d.nr;
    out->nt = v.nt;
    out->np = v.np;
    out->n = v.n;
    out->dg = v.dg;
    out->ar = v.ar;
    out->at = v.at;
    out->ap = v.ap;
    out->w = v.w;
    out->im = v.im;
    out->cp = v.cp;
    out->q = v.q;
    out->g = v.g;
    out->rho = v.rho;
    out->kap = v.kap;
    return RT_OK;
}

rt_status rt_rosseland_depth(rt_ctx *ctx, const rt_opacity *op, const double *rho, const double *T, double *tau_R)
{
    if (!ctx) return fail(nullptr, RT_EINVAL, "context is NULL");
    if (op) { rt_status s = rt_set_opacity(ctx, op); if (s) return s; }
    RT_CHECK(ctx, ctx->have_opac, "no opacity table on the context");
    RT_CHECK(ctx, rho && T && tau_R, "rt_rosseland_depth: NULL field pointer");
    launch_tau_rosseland(ctx->d, ctx->op, ctx->geo.rf, rho, T, tau_R, ctx->stream);
    RT_HIP(ctx, hipGetLastError());
    return RT_OK;
}

rt_status rt_relax(rt_ctx *ctx, const rt_opacity *op, const rt_star *st, const rt_fld_params *p,
                   const rt_solve_opts *o, const double *rho, double *T, double *E, double tol_change,
                   int max_steps, rt_relax_stats *stats)
{
    if (!ctx) return fail(nullptr, RT_EINVAL, "context is NULL");
    RT_CHECK(ctx, rho && T && E && o && p, "rt_relax: NULL argument");
    RT_CHECK(ctx, tol_change > 0.0 && isfin(tol_change), "tol_change must be positive");
    RT_CHECK(ctx, max_steps > 0, "max_steps must be positive");
    const long n = ctx->d.n;
    if (!ctx->Tn) {
        ctx->Tn = dalloc<double>(ctx, n);
        if (!ctx->Tn) return fail(ctx, RT_ENOMEM, "rt_relax: out of device memory");
    }
    rt_relax_stats local{};
    rt_relax_stats *R = stats ? stats : &local;
    *R = rt_relax_stats{};
    R->last_change = INFINITY;
    Clock clk;
    hipStream_t s = ctx->stream;
    rt_status status = RT_OK;
    DevScalars *h = ctx->h_sc;
    // steps replayed from one captured graph where they can be (see step_graph_applies)
    struct GraphGuard {
        hipGraphExec_t g = nullptr;
        ~GraphGuard() { if (g) (void)hipGraphExecDestroy(g); }
    } guard;
    hipGraphExec_t &gx = guard.g;
    if (step_graph_applies(ctx, o)) {
        if (op) { rt_status e = rt_set_opacity(ctx, op); if (e) return e; }
        if (st) { rt_status e = rt_set_star(ctx, st); if (e) return e; }
        RT_CHECK(ctx, ctx->have_opac, "no opacity table on the context");
        RT_CHECK(ctx, ctx->have_star, "no star on the context");
        if (rt_status e = check_fld(ctx, p)) return e;
        if (rt_status e = capture_step(ctx, p, o, rho, T, E, &gx)) return e;
    }
    for (int k = 0; k < max_steps; k++) {
        rt_step_stats ss{};
        bool replayed = false;
        if (gx) {
            RT_HIP(ctx, hipEventRecord(ctx->ev[0], s));
            RT_HIP(ctx, hipGraphLaunch(gx, s));
            RT_HIP(ctx, hipEventRecord(ctx->ev[5], s));
            if (rt_status e = read_scalars(ctx)) return e;
            if (step_graph_result_ok(h, o)) {
                replayed = true;
                float t05 = 0.0f;
                (void)hipEventElapsedTime(&t05, ctx->ev[0], ctx->ev[5]);
                ss.ms_total = t05;
                if (o->mode != RT_SOLVE_NONE) {
                    ss.solve.iters = h->iters;
                    ss.solve.relres = std::sqrt(h->res2 / h->bnorm2);
                    ss.solve.reduced = 1;
                }
            } else {
                // the host-driven path decides this step: from the saved temperature,
                // with directions as after a failed solve
                RT_HIP(ctx, hipMemcpyAsync(T, ctx->Tn, n * sizeof(double), hipMemcpyDeviceToDevice, s));
                if (rt_status e = reset_directions(ctx)) return e;
            }
        }
        if (!replayed) {
            RT_HIP(ctx, hipMemcpyAsync(ctx->Tn, T, n * sizeof(double), hipMemcpyDeviceToDevice, s));
            // the tables are uploaded by the first step only
            const bool first = k == 0 && !gx;
            status = rt_step(ctx, first ? op : nullptr, first ? st : nullptr, p, o, rho, T, E, nullptr, &ss);
        }
        R->steps = k + 1;
        R->krylov_iters += ss.solve.iters;
        R->ms_device += ss.ms_total;
        R->last = ss;
        if (status != RT_OK) break;
        if (!replayed) {
            double *dchange = reinterpret_cast<double *>(reinterpret_cast<char *>(ctx->sc) + offsetof(DevScalars, change));
            launch_max_change(n, ctx->nblk, T, ctx->Tn, ctx->partials, ctx->counter, dchange, s);
            RT_HIP(ctx, hipGetLastError());
            if (rt_status e = read_scalars(ctx)) return e;
        }
        R->last_change = h->change;
        if (!isfin(R->last_change)) {
            status = fail(ctx, RT_ENONFINITE, "rt_relax: non-finite temperature");
            break;
        }
        if (R->last_change < tol_change) break;
    }
    R->ms = clk.ms();
    if (status != RT_OK) return status;
    if (!(R->last_change < tol_change)) return fail(ctx, RT_ENOCONV, "rt_relax: max_steps reached");
    return RT_OK;
}

}  // extern "C"
