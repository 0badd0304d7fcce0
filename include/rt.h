/*
 * rt.h - C-ABI of librtmi, the MI355X (gfx950) radiation step of Kuiper et al.,
 * "Fast and accurate frequency dependent radiation transport for hydrodynamics
 * simulations in massive star formation".
 *
 * One call of rt_step is one pass of the main loop of the paper's Fig. 1:
 * frequency-dependent ray trace of the stellar irradiation (Eqs. 17-20), radiation
 * energy E^n from Eq. (16), implicit gray FLD solve for E^{n+1} (Eqs. 8-15), Newton
 * update of the temperature (Eq. 16), and the radiative force (Eqs. 27-36).
 *
 * Conventions (all entry points):
 *  - Grid: spherical-polar, N_r x N_theta x N_phi cells.  Cell (i, j, k) is stored at
 *    c = i + N_r (j + N_theta k) (r fastest).  Radial face i (at r_face[i],
 *    i = 0..N_r) of column (j, k) is stored at i + (N_r + 1)(j + N_theta k).
 *  - Field arguments (rho, T, E, ...) are DEVICE pointers to contiguous float64 arrays
 *    in that layout, owned by the caller; the library never frees or retains them.
 *  - rt_grid / rt_opacity / rt_star describe the problem with HOST arrays that are
 *    copied by the call that receives them.
 *  - All work is enqueued on the stream given to rt_create; calls return once the
 *    work is enqueued, except where a call states that it synchronises (solves read
 *    their convergence scalars back to the host).
 *  - Units are CGS.  No exception crosses the ABI; a failing call returns a non-zero
 *    rt_status and rt_last_error(ctx) describes it.  Arguments are validated on the
 *    host before anything is launched.
 *  - A context is used by one host thread at a time.
 */
#ifndef RTMI_RT_H
#define RTMI_RT_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RT_OK = 0,
    RT_EINVAL = 1,     /* bad argument (size, NULL, inconsistent table) */
    RT_EDEVICE = 2,    /* HIP runtime error */
    RT_ENOMEM = 3,     /* device allocation failed */
    RT_ENONFINITE = 4, /* NaN/Inf met in a residual or norm */
    RT_ENOCONV = 5     /* iteration limit reached; outputs hold the last iterate */
} rt_status;

typedef struct rt_ctx rt_ctx;

/* Grid faces (host arrays): r_face[nr+1] increasing and > 0, th_face[nt+1] within
 * [0, pi], ph_face[np+1] increasing; phi is periodic over [ph_face[0], ph_face[np]]. */
typedef struct {
    int nr, nt, np;
    const double *r_face, *th_face, *ph_face;
} rt_grid;

/* Opacity table (host arrays), Sect. "Frequency dependent irradiation": kappa[n_T][n_nu]
 * is kappa_nu at the bin mid-frequencies nu[n_nu] for the temperatures T[n_T]
 * (increasing); kappa_P / kappa_R are the Planck / Rosseland means at T[] (> 0).
 * kappa_nu is interpolated linearly in T, the means log-log; values are clamped to
 * the end nodes outside the table.  1 <= n_nu <= 64, 2 <= n_T <= 128. */
typedef struct {
    int n_T, n_nu;
    const double *T, *nu, *kappa, *kappa_P, *kappa_R;
} rt_opacity;

/* Central star: radius, effective temperature and the flux per bin at the stellar
 * surface, F_nu[n_nu] (host array, erg s^-1 cm^-2), e.g. from rt_star_bin_flux. */
typedef struct {
    double R_star, T_star;
    const double *F_nu;
} rt_star;

/* Parameters of the implicit FLD step (Eqs. 9, 15, 16): time step dt [s], specific
 * heat c_V [erg g^-1 K^-1], outer Dirichlet temperature T_bc [K] (E = a T_bc^4 in a
 * ghost cell beyond the last radial face; zero flux through the inner radial face and
 * the poles; phi periodic), and the floor applied to E^n. */
typedef struct {
    double dt, c_V, T_bc, E_floor;
} rt_fld_params;

/* Device view of the assembled Jacobi-scaled system A^ y = b^ (unit diagonal, A^ =
 * S A S with S = diag(d)^-1/2, E = s * y).  Pointers are owned by the context and stay
 * valid until the next rt_fld_assemble / rt_step / rt_destroy. */
typedef struct {
    long n;
    const double *ahat;   /* [3][n] scaled off-diagonals of the outward r, theta, phi faces */
    const float *ahat32;  /* [3][n] the same in float32 (inner solves of the mixed mode) */
    const double *s;      /* [n] Jacobi scale d^-1/2 */
    const double *bhat;   /* [n] scaled right-hand side */
    const double *w;      /* [3][n] unscaled outward face weights A_f D_f / ds_f; the radial
                             weight of the last cell is the Dirichlet face */
    const double *chi;    /* [n] kappa_R(T^n) rho */
} rt_system;

typedef enum {
    RT_SOLVE_FP64 = 0,    /* CG on A^ in float64 (the plain method; also the fallback) */
    RT_SOLVE_MIXED = 1,   /* float64 iterative refinement around float32 inner CG; when a
                             float32 cycle needs over 2048 iterations for a tenfold drop,
                             or two cycles fail to halve the true residual (cond(A^) too
                             large for float32), float64 CG finishes (fallback = 1) */
    RT_SOLVE_LEARNED = 2, /* a Krylov method preconditioned by a network (flexible CG with
                             float64 refinement, or flexible GMRES: see inner), then the
                             planned finish once inner_max_iter applications are spent */
    RT_SOLVE_GMRES = 3,   /* restarted GMRES(m) on A^ in float64 (the paper's solver class,
                             Sect. "The generalized minimal residual method"; m = restart) */
    RT_SOLVE_NONE = 4     /* no diffusion: E^{n+1} = a T_bc^4 of the assembled system in every
                             cell (the runs without FLD of the run table, where the thermal
                             field is never transported); no other option is read */
} rt_solve_mode;

typedef struct rt_net rt_net;

typedef struct {
    int mode;            /* rt_solve_mode */
    double tol;          /* stop when ||b^ - A^ y|| / ||b^|| <= tol (float64, true residual) */
    int max_iter;        /* limit on (inner) Krylov iterations in total */
    int check_every;     /* iterations between host convergence polls (default 32; the
                            one-workgroup solve of RT_LAUNCH_BLOCK checks on the device) */
    double inner_tol;    /* relative reduction asked of each inner solve (mixed / learned) */
    int inner_max_iter;  /* limit per inner solve */
    rt_net *net;         /* network for RT_SOLVE_LEARNED, else NULL */
    int restart;         /* RT_SOLVE_GMRES: Krylov steps per cycle, 1..63 (<= 0: 30) */
    int reduce;          /* RT_SOLVE_FP64 / RT_SOLVE_MIXED: 1 = eliminate the red cells of the
                            red-black colouring ((i + j + k) odd) and run CG on the Schur
                            complement S = I - B^T B over the black cells, then recover the
                            red ones (the same solution and stopping test, about half the
                            iterations at the same bytes each); used when N_r is even and
                            N_phi is even or 1, else the full system is solved.
                            RT_SOLVE_LEARNED: 1 = the finish after the network budget is
                            the reduced mixed solve instead of full-system float64 CG */
    int precond;         /* without reduce: 0 = the Jacobi scaling alone (the default),
                            1 (RT_SOLVE_FP64) = CG preconditioned by the radial-line block
                            Jacobi: each radial row's tridiagonal block of A^ solved exactly
                            (the block-Jacobi class of the paper's solver set-up, Sect.
                            "Numerical setup", as a comparator), 2 = one multigrid cycle per
                            iteration (an extension, not in the paper: see rt_mg_apply):
                            RT_SOLVE_FP64 runs float64 CG with it (check_every defaults to 8
                            there), RT_SOLVE_MIXED flexible CG in float32 with float64 dots
                            and reliable updates (a non-finite float32 state hands over to
                            the float64 form: fallback = 1) */
    int launch;          /* rt_launch: how the CG iterations of RT_SOLVE_FP64 / RT_SOLVE_MIXED
                            (reduced or not) reach the GPU; every choice computes the same
                            method, DIRECT and GRAPH bit for bit alike */
    int inner;           /* rt_inner: the Krylov method of RT_SOLVE_LEARNED */
    int cycle;           /* precond = 2: 0 = the coarse corrections of levels 1 to 3 are two
                            flexible-CG steps each (K-cycle, the default), 1 = plain V-cycle
                            (cheaper per iteration, more iterations), n = 2..8: K-cycle
                            steps on levels 1 to n (each level deeper doubles the visits to
                            the levels below it) */
} rt_solve_opts;

typedef enum {
    RT_INNER_FCG = 0,     /* flexible CG in float32 (Notay's FCG with one A-orthogonalisation)
                             with float64 dots and reliable updates */
    RT_INNER_FGMRES = 1   /* flexible GMRES(m) (Saad), m = restart: each Arnoldi step applies
                             the network to the float32-rounded basis vector and keeps its
                             answer z_j in a second basis; the Arnoldi process and the update
                             y += Z z are float64.  One network application per iteration; a
                             cycle that runs out of applications is closed with the steps
                             taken, then the planned finish runs */
} rt_inner;

typedef enum {
    RT_LAUNCH_AUTO = 0,   /* BLOCK where it applies, else GRAPH on grids of at most 4,194,304
                             cells (where launches dominate), else DIRECT; in rt_relax, with
                             BLOCK, whole steps are replayed from one HIP graph */
    RT_LAUNCH_DIRECT = 1, /* every kernel launched from the host; the only choice that samples
                             the kernel times of rt_solve_stats */
    RT_LAUNCH_GRAPH = 2,  /* the chunks of iterations between convergence polls replayed from
                             HIP graphs captured once per context */
    RT_LAUNCH_BLOCK = 3   /* reduced float64 CG (reduce = 1, also where a reduced mixed solve
                             falls back to it) with at most 2048 black cells: all
                             iterations inside one workgroup, the vectors whose neighbours are
                             read kept in LDS (dot products summed in another order than the
                             multi-block kernels); other solves as AUTO */
} rt_launch;

typedef struct {
    int status;          /* rt_status of the solve */
    int iters;           /* Krylov iterations (inner iterations in mixed / learned modes) */
    int outer_iters;     /* float64 refinement steps (mixed / learned) */
    int precond_applies; /* network applications (learned) */
    int fallback;        /* 1 if a mixed solve's precision guard, or a learned solve's
                            non-finite network output, handed the solve to the float64
                            method (a failure of the faster method, not a wrong answer) */
    double relres;       /* final true relative residual, computed in float64 */
    double ms;           /* wall time of the solve (host clock, includes polls) */
    double ms_dir;       /* mean device time of one direction+operator kernel (sampled once per poll) */
    double ms_upd;       /* mean device time of one update kernel (sampled likewise) */
    int kernel_samples;  /* number of samples behind ms_dir / ms_upd */
    int reduced;         /* 1 if the red-black reduced system was solved (iters count its
                            iterations; ms_dir then covers its red and black passes) */
    double ms_black;     /* reduced solves: mean device time of the black pass alone (ms_dir -
                            ms_black is the red pass); precond = 1 or 2: the direction
                            kernel alone (ms_dir - ms_black is the block solve or the
                            V-cycle) */
    int handover;        /* learned solves: 1 if the network budget (inner_max_iter
                            applications) ran out above tol and the planned finish (float64
                            CG, or the reduced mixed solve with reduce = 1) completed it */
} rt_solve_stats;

typedef struct {
    rt_solve_stats solve;
    double ms_raytrace, ms_assemble, ms_solve, ms_newton, ms_total; /* device-event times */
} rt_step_stats;

/* ------------------------------------------------------------------ context */

/* Creates a context for grid g and n_nu frequency bins, enqueuing on `stream`
 * (a hipStream_t; NULL = the default stream).  Allocates every workspace of the
 * radiation step (about 30 float64-equivalents per cell).  Select the device first
 * (hipSetDevice); the context stays on it.  RT_EINVAL for N_r > 2944 (the ray trace's
 * face flux keeps one radial factor per cell of a column in LDS beside the opacity table). */
rt_status rt_create(rt_ctx **out, const rt_grid *g, int n_nu, void *stream);
void rt_destroy(rt_ctx *ctx);
/* Message of the last failing call on ctx (or of the last failing rt_create when ctx
 * is NULL).  Valid until the next call. */
const char *rt_last_error(const rt_ctx *ctx);
/* Number of cells of the context's grid. */
long rt_ncell(const rt_ctx *ctx);

/* Eq. (20): flux of each frequency bin at the stellar surface, pi * int B_nu(T_star)
 * d nu over the bin, whose edges are the midpoints between neighbouring mid-frequencies
 * (0 and infinity at the ends), so the bins sum to sigma T_star^4 (Eq. 18).  Host
 * arrays nu[n_nu] (increasing) and F_out[n_nu]. */
rt_status rt_star_bin_flux(double T_star, int n_nu, const double *nu, double *F_out);

/* Uploads the opacity table / stellar spectrum to the context (they are also taken by
 * the calls below when their pointer argument is not NULL). */
rt_status rt_set_opacity(rt_ctx *ctx, const rt_opacity *op);
rt_status rt_set_star(rt_ctx *ctx, const rt_star *st);

/* ------------------------------------------------------------ the step's calls */

/* Ray trace (Eqs. 17-20, optical depth zero at the inner radial face).  Per radial
 * column and bin: tau_nu grows by kappa_nu(T_i) rho_i dr_i through cell i (float64
 * accumulation), F_nu(r) = F_nu(R_*) (R_* / r)^2 exp(-tau_nu).  Outputs (device):
 *   q_star[n]  absorbed stellar power per volume, (A_- F_- - A_+ F_+)/V summed over
 *              bins (the cell-integrated form of Eqs. 28-33, 36);
 *   S_abs[n]   sum_nu kappa_nu Fbar_nu / c = q_nu / (rho c), the irradiation term of
 *              Eq. (16) in the frequency-dependent form;
 *   F_face     total stellar flux at every radial face, (N_r+1) N_theta N_phi, or NULL;
 *   F_face_nu  the flux of every bin at every radial face, F_nu(R_star) (R_star / r)^2 e^-tau_nu
 *              (Eqs. 17, 19), (N_r+1) N_theta N_phi n_nu with the bin fastest:
 *              F_face_nu[f * n_nu + b] for the face index f of F_face; or NULL (it is
 *              n_nu times the size of F_face: 34 GB at 512x256x512 with 64 bins).
 * Without F_face and F_face_nu the mapping is chosen by the column length (see
 * rt_raytrace_mapped); with either, q_star and S_abs come from lanes on bins.
 * op / st may be NULL to use the tables already on the context. */
rt_status rt_raytrace(rt_ctx *ctx, const rt_opacity *op, const rt_star *st,
                      const double *rho, const double *T, double *q_star, double *S_abs,
                      double *F_face, double *F_face_nu);

/* The two mappings of a radial column onto a 64-lane wavefront for q_star and S_abs
 * (Eqs. 17-20 and 28-36, the definitions and device arrays of rt_raytrace):
 *   RT_LANES_BINS   lanes on frequency bins, each walking the column cell by cell (the
 *                   float64 transmission product in the oracle's order), the bin sums by
 *                   a transpose through LDS;
 *   RT_LANES_CELLS  lanes on radial cells (8 per lane, segments of 512 cells), the
 *                   transmissions of each bin multiplied across the lanes by a scan, the
 *                   sum over bins kept per cell.
 * rt_raytrace without face fluxes uses RT_LANES_CELLS where the column fills its
 * 512-cell segments to 90 % or more (it is the faster there), else RT_LANES_BINS; the
 * face fluxes always come from RT_LANES_BINS.  The two agree up to the order of the
 * float64 products and sums. */
typedef enum { RT_LANES_BINS = 0, RT_LANES_CELLS = 1 } rt_raytrace_mapping;

/* q_star and S_abs with the given mapping (to time the two against each other).  Uses the
 * context's opacity table and star; RT_EINVAL if either is missing, a pointer is NULL or
 * mapping is not an rt_raytrace_mapping. */
rt_status rt_raytrace_mapped(rt_ctx *ctx, int mapping, const double *rho, const double *T, double *q_star,
                             double *S_abs);

/* Fig. 1 "Radiation Energy": E[n] = max(a T^4 - S_abs / kappa_P(T), E_floor). */
rt_status rt_energy(rt_ctx *ctx, const rt_opacity *op, const rt_fld_params *p,
                    const double *T, const double *S_abs, double *E);

/* Backward-Euler finite-volume form of Eq. (15):
 *   V/(dt f_c) (E - E^n) = sum_faces w_f (E_nb - E) + V (q_star + Q_plus),
 * f_c from Eq. (9), w_f = A_f D_f / ds_f with D from Eqs. (11)-(13) at each face
 * (kappa_R rho and E arithmetic means of the two cells, coefficients at (E^n, T^n)).
 * Writes the Jacobi-scaled system into the context; *sys receives its device view.
 * Q_plus may be NULL (static problem). */
rt_status rt_fld_assemble(rt_ctx *ctx, const rt_opacity *op, const rt_fld_params *p,
                          const double *rho, const double *T, const double *E_n,
                          const double *q_star, const double *Q_plus, rt_system *sys);

/* y = A^ x with the context's current system (float64), device arrays of n. */
rt_status rt_spmv(rt_ctx *ctx, const double *x, double *y);

/* Implicit solve of the assembled system (the paper's implicit Krylov step).  E holds
 * the start value on entry (normally E^n) and E^{n+1} = s * y on exit.  Synchronises
 * with the stream to poll convergence.  Returns RT_ENOCONV (E still written) when the
 * iteration limit is met, RT_ENONFINITE on NaN/Inf. */
rt_status rt_fld_solve(rt_ctx *ctx, const rt_solve_opts *o, double *E, rt_solve_stats *st);

/* Newton-Raphson on Eq. (16), a T^4 = E + S_abs / kappa_P(T), per cell; T holds the
 * start value (T^n) on entry and the root on exit.  The root returned is the smallest
 * one (the table's sublimation drop can make Eq. (16) non-monotone). */
rt_status rt_temperature(rt_ctx *ctx, const rt_opacity *op, const double *E,
                         const double *S_abs, double *T);

/* Radiative force density (Eq. 27) per cell, f[4][n] (device): component 0 is the
 * stellar part q_star / c (Eq. 36 in the cell-integrated form of Eq. 33); 1-3 are the
 * thermal part kappa_R rho F / c along r, theta, phi, with the FLD flux F = -D grad E
 * (Eq. 10) of the context's current system evaluated at the faces with E and averaged
 * over the two faces of each direction. */
rt_status rt_force(rt_ctx *ctx, const double *E, const double *q_star, double *f);

/* One main-loop pass of Fig. 1 for the given density: rt_raytrace(rho, T^n) ->
 * rt_energy -> rt_fld_assemble -> rt_fld_solve (start E^n) -> rt_temperature ->
 * rt_force.  T: T^n in, T^{n+1} out.  E: E^{n+1} out.  f_rad (4 n) may be NULL.
 * The stellar quantities of the step stay on the context (rt_step_fields). */
rt_status rt_step(rt_ctx *ctx, const rt_opacity *op, const rt_star *st,
                  const rt_fld_params *p, const rt_solve_opts *o, const double *rho,
                  double *T, double *E, double *f_rad, rt_step_stats *stats);

/* Device views of the last step's q_star, S_abs and E^n (n each). */
rt_status rt_step_fields(rt_ctx *ctx, const double **q_star, const double **S_abs,
                         const double **E_n);

/* ------------------------------------------------------------ the main iteration */

/* Gray irradiation (Eqs. 18, 19): the one-bin table whose opacity at each table
 * temperature is the F_nu-weighted mean of the bins, sum_b kappa[k][b] F_nu[b] /
 * sum_b F_nu[b] (the Planck mean at T_* when F_nu comes from rt_star_bin_flux, keeping
 * the table's dust-temperature dependence), and the total flux sum_b F_nu[b] (sigma
 * T_*^4).  Host arrays: op's table, F_nu[n_nu] (>= 0, positive sum), kappa_gray[n_T]
 * out; *F_total out; *nu_gray (may be NULL) the flux-weighted mean frequency.  A
 * context created with n_nu = 1 and given {kappa_gray} with that star flux runs the
 * gray variant of every call above.  Host computation, no device work. */
rt_status rt_gray_table(const rt_opacity *op, const double *F_nu, double *kappa_gray, double *F_total,
                        double *nu_gray);

/* z = M^-1 r for the radial-line block-Jacobi preconditioner of the current system
 * (precond = 1): per radial row, the tridiagonal block of A^ (unit diagonal, the radial
 * off-diagonals) solved exactly.  Device arrays of n; r and z must not overlap. */
rt_status rt_precond_apply(rt_ctx *ctx, const double *r, double *z);

/* The multigrid preconditioner of precond = 2 (an extension of the implicit solve of
 * Eq. 15, not in the paper): z = M_mg r, one cycle for the current system, with the
 * K-cycle steps of cycle = 0 (levels 1 to 3, the solver's default).  Levels:
 * A_0 = A^; A_(l+1) = P_l^T A_l P_l over aggregates of 1 x 2 x 2 cells (theta and phi
 * pairs merged, the radius kept; a lone last row where a size is odd), with P_l[f, C] =
 * B_f / Bc_C, B_0 = 1/s and Bc_C^2 the sum of B_f^2 over the aggregate; the last level
 * is one radial line, solved exactly.  Smoother: x <- x + 0.8 M^-1 (b - A x), M the
 * diagonal and phi couplings of each (r, theta) line (periodic).  Cycle: pre-smoothing
 * from 0, restriction of the residual by P^T, the coarse correction, prolongation by P,
 * post-smoothing; the coarse correction is the cycle one level down (V-cycle), or on
 * levels 1 to 3 two flexible-CG steps preconditioned by the cycle from that level
 * (K-cycle: x = a_1 z_1 + a_2 (z_2 + beta z_1), beta = -(z_2.A z_1)/(z_1.A z_1), a =
 * p.r / p.A p), which makes the preconditioner nonlinear: the solver's outer CG is the
 * flexible one.  Float32 inside, set-up in float64 once per assembled system.  Device
 * arrays of n; r and z must not overlap.  The hierarchy is allocated at the first use
 * (about 100 bytes per cell). */
rt_status rt_mg_apply(rt_ctx *ctx, const double *r, double *z);

/* Device view of level `level` (0 = finest) of the current system's multigrid hierarchy
 * (set up if needed): its sizes and float32 arrays in the field layout (r fastest, then
 * theta, then phi) of that level.  dg is NULL on level 0 (unit diagonal), where ar / at /
 * ap are A^'s float32 couplings; w (prolongation weights to the next level), the phi-line
 * factors im, cp, q, g (per cell) and rho, kap (per (r, theta) line) are NULL on the last
 * level.  Valid until the next assembly or rt_destroy. */
typedef struct {
    int levels;  /* number of levels */
    int nr, nt, np;
    long n;
    const float *dg, *ar, *at, *ap;
    const float *w;
    const float *im, *cp, *q, *g;
    const float *rho, *kap;
} rt_mg_level_view;
rt_status rt_mg_level(rt_ctx *ctx, int level, rt_mg_level_view *out);

/* Diagnostic of Sect. "The Flux Limited Diffusion approximation" (Fig. 8): the optical
 * depth of the thermal emission integrated inward from the outer edge along each radial
 * ray, tau_R = sum of kappa_R(T) rho (r_{i+1} - r_i) over the cells between a radial
 * face and r_out.  Device arrays rho[n], T[n] in, tau_R[(N_r + 1) N_theta N_phi] out at
 * the radial faces (face layout of rt_raytrace's F_face; 0 at r_out).  op may be NULL
 * to use the context's table. */
rt_status rt_rosseland_depth(rt_ctx *ctx, const rt_opacity *op, const double *rho, const double *T, double *tau_R);

typedef struct {
    int steps;           /* main iterations taken */
    double last_change;  /* largest relative temperature change of the last step */
    long krylov_iters;   /* Krylov iterations summed over the steps */
    double ms;           /* host wall time of the call */
    double ms_device;    /* device time of the steps (sum of their ms_total) */
    rt_step_stats last;  /* statistics of the last step */
} rt_relax_stats;

/* The main loop of Fig. 1 run to a steady state (Sect. "Numerical setup": the loop stops
 * when the temperature of every cell changes by less than 0.01 % in one step, i.e.
 * tol_change = 1e-4): rt_step until max_c |T^{n+1}_c - T^n_c| / T^n_c < tol_change or
 * max_steps steps.  T: start temperature in, the last iterate out; E: E^{n+1} of the
 * last step.  o->mode = RT_SOLVE_NONE runs the loop without diffusion.  Synchronises
 * once per step to read the change back.  With o->launch = RT_LAUNCH_AUTO, a loop whose
 * steps solve with the reduced float64 CG in one workgroup (RT_SOLVE_FP64, reduce = 1,
 * at most 2048 black cells), or without diffusion, captures one step in a HIP graph at
 * the start of the call and replays it every step (the solver's set-up on the device, one
 * read-back per step); a step the replay cannot finish as the host-driven step would (a
 * non-finite value, an iteration limit, a true residual above tol) is redone from its
 * start temperature on that path, so the results are the same bits as with
 * RT_LAUNCH_BLOCK, which launches every step from the host.  Returns RT_ENOCONV when max_steps pass
 * without reaching tol_change or a step's solve hits its limit (outputs hold the last
 * iterate), RT_ENONFINITE for a non-finite temperature.  Allocates one float64 field
 * on the context at its first call. */
rt_status rt_relax(rt_ctx *ctx, const rt_opacity *op, const rt_star *st, const rt_fld_params *p,
                   const rt_solve_opts *o, const double *rho, double *T, double *E, double tol_change,
                   int max_steps, rt_relax_stats *stats);

/* ------------------------------------------------ learned preconditioner (network) */

/* The network is a 3-level 3-D convolutional U-Net (3x3x3 kernels, 16/32/64 channels,
 * average pooling, nearest-neighbour upsampling with skip concatenation, ReLU, a final
 * 1x1 convolution), evaluated and trained in bf16 on the matrix cores with fp32
 * accumulation and fp32 master weights.  Its input has 16 channels per cell: the
 * residual scaled to unit RMS, three operator features (log10 of minus the scaled
 * off-diagonals of the outward faces, clipped to [-30, 0] and mapped to [-1, 1]) and
 * zeros; its output approximates the scaled error A^-1 r.  Convolutions pad with zeros
 * in r and theta and wrap in phi; grid dimensions must be divisible by 4.  Tensors are
 * channels-last: x[c * C + ch].  Weights of layer l are w[(tap * Cout + co) * Cin + ci]
 * with tap = (dk+1)*9 + (dj+1)*3 + (di+1); all parameters form one flat fp32 vector
 * [w_0, b_0, w_1, b_1, ...]. */
typedef struct {
    unsigned seed; /* initialisation seed (counter-based hash, He-uniform weights) */
} rt_net_config;

/* Creates a network on the current device. */
rt_status rt_net_create(const rt_net_config *cfg, rt_net **out);
void rt_net_destroy(rt_net *net);
const char *rt_net_last_error(const rt_net *net);
long rt_net_param_count(const rt_net *net);
/* Host copies of the fp32 master parameters / of the last gradient (n = param count). */
rt_status rt_net_get_params(const rt_net *net, float *host, long n);
rt_status rt_net_get_grads(const rt_net *net, float *host, long n);
/* Replaces the parameters (resets the Adam state). */
rt_status rt_net_set_params(rt_net *net, const float *host, long n);
rt_status rt_net_save(const rt_net *net, const char *path);
rt_status rt_net_load(rt_net *net, const char *path);

/* z[n] (fp32, device) = network(X) for X[n][16] (bf16 bits, device) on the context's grid. */
rt_status rt_net_forward(rt_ctx *ctx, rt_net *net, const void *X, float *z);
/* The learned preconditioner's action z = M(r) as RT_SOLVE_LEARNED applies it: the
 * residual r[n] (fp32, device) scaled to unit RMS and the operator features of the
 * context's assembled system form the input, and the output is scaled back by the same
 * factor (z[n], fp32, device).  Needs an assembled system (RT_EINVAL otherwise) and grid
 * dimensions divisible by 4; overwrites the context's Krylov scalars, so not during a
 * solve on the same context. */
rt_status rt_net_apply(rt_ctx *ctx, rt_net *net, const float *r, float *z);
/* Forward pass, loss L = ||z - e||^2 / ||e||^2 for the target e[n] (fp32, device) and
 * backward pass; the gradient stays on the network for rt_net_adam.  z (device) and
 * loss (host) may be NULL. */
rt_status rt_net_loss_grad(rt_ctx *ctx, rt_net *net, const void *X, const float *e, float *z, double *loss);
/* Residual loss of a preconditioner: L = ||A z - r||^2 / ||r||^2 with z = network(X),
 * for the residual r[n] (fp32, device; normally the unit-RMS residual that channel 0 of
 * X encodes) and the scaled operator a32[3n] (fp32, device, the layout of
 * rt_system.ahat32: radial, polar and azimuthal outward coefficients per cell), then
 * the backward pass with dL/dz = 2 A (A z - r) / ||r||^2 (A is symmetric).  The
 * gradient stays on the network; z and loss may be NULL. */
rt_status rt_net_loss_grad_resid(rt_ctx *ctx, rt_net *net, const void *X, const float *r, const float *a32, float *z,
                                 double *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with learning rate lr. */
rt_status rt_net_adam(rt_ctx *ctx, rt_net *net, double lr);

/* Training pairs (residual -> error) made by the float64 method itself on the
 * context's grid: rt_dataset_add runs float64 CG on the context's current system from
 * E0 (device, E-space start value, normally E^n) to a relative residual of 1e-12 for
 * the reference y*, then, for each iteration count k in iters, k CG iterations from
 * E0 give y_k; the pair is (r_k = b - A y_k, e_k = y* - y_k), both scaled by
 * sqrt(n) / ||r_k||, stored with the system's operator features and (once per call)
 * a float32 copy of the scaled operator for the residual loss.  Returns RT_EINVAL
 * when the set is full. */
typedef struct rt_dataset rt_dataset;
rt_status rt_dataset_create(rt_ctx *ctx, int capacity, rt_dataset **out);
void rt_dataset_destroy(rt_dataset *ds);
int rt_dataset_size(const rt_dataset *ds);
rt_status rt_dataset_add(rt_ctx *ctx, rt_dataset *ds, const double *E0, const int *iters, int n_iters);
/* Like rt_dataset_add, but y_k comes from k iterations of the learned flexible CG with
 * the network net (no float64 fallback): pairs from the residuals that the learned
 * solver itself produces, whose distribution differs from that of the plain CG
 * iterates (training on both is what makes the network a usable preconditioner). */
rt_status rt_dataset_add_learned(rt_ctx *ctx, rt_dataset *ds, rt_net *net, const double *E0, const int *iters,
                                 int n_iters);

typedef enum {
    RT_LOSS_ERROR = 0,    /* ||z - e||^2 / ||e||^2 against the CG error e_k */
    RT_LOSS_RESIDUAL = 1  /* ||A z - r||^2 / ||r||^2 (rt_net_loss_grad_resid) */
} rt_loss;
typedef struct {
    int epochs;   /* passes over the set */
    double lr;    /* peak learning rate (cosine decay to lr/10 over the run) */
    unsigned seed; /* order of the pairs in each epoch */
    int loss;     /* rt_loss */
} rt_train_opts;
typedef struct {
    int steps;
    double loss_first_epoch, loss_last_epoch; /* mean loss of the first / last epoch */
    double ms;
} rt_train_stats;
/* Trains the network on the set (one pair per Adam step), on the context's stream. */
rt_status rt_net_train(rt_ctx *ctx, rt_net *net, rt_dataset *ds, const rt_train_opts *o, rt_train_stats *st);

/* Layer-level building blocks (bf16 tensors as raw 16-bit values, device pointers,
 * enqueued on `stream`).  Forward: y = act(conv3x3x3([up?(x1), x2], w) + bias), x1 with
 * c1 channels on the level of y (up1 = 0) or on the 2x coarser level read through
 * nearest-neighbour upsampling (up1 = 1), x2 with c2 channels (may be 0); outputs bf16
 * y and/or fp32 yf (either may be NULL); c1, c2, cout multiples of 16, cout <= 64.  The
 * convolutions (and the network) take grids of fewer than 2^31 cells (RT_EINVAL). */
rt_status rt_nn_conv3d_fwd(void *stream, int nr, int nt, int np, const void *x1, int c1, int up1, const void *x2,
                           int c2, const void *w, const float *bias, int cout, int relu, void *y, float *yf);
/* The U-Net's pooled layer in one pass: y = relu(conv3x3x3(x, w) + bias) with 16 input
 * and 16 output channels (bf16 y[nr nt np][16]) and its 2x2x2 average pool on the 2x
 * coarser level (bf16 yp[nr/2 nt/2 np/2][16], the children summed in fp32 in the order
 * r, theta, phi); the same bits as rt_nn_conv3d_fwd followed by that pooling.  nr, nt,
 * np even (RT_EINVAL otherwise, or for a NULL pointer). */
rt_status rt_nn_conv3d_fwd_pool(void *stream, int nr, int nt, int np, const void *x, const void *w, const float *bias,
                                void *y, void *yp);
/* Data gradient: d[x1|x2] = conv^T(dy masked by yrelu > 0 when yrelu != NULL) with the
 * transposed weights wt[(tap * Cin + ci) * Cout + co]; fp32 outputs on the level of dy
 * (for an upsampled x1, the gradient of the upsampled tensor). */
rt_status rt_nn_conv3d_bwd_data(void *stream, int nr, int nt, int np, const float *dy, const void *yrelu, int cout,
                                const void *wt, int c1, float *d1, int c2, float *d2);
/* Weight and bias gradients (fp32, dw[27][cout][c1+c2], db[cout]); cout <= 64; synchronises. */
rt_status rt_nn_conv3d_bwd_weight(void *stream, int nr, int nt, int np, const float *dy, const void *yrelu, int cout,
                                  const void *x1, int c1, int up1, const void *x2, int c2, float *dw, float *db);
/* rt_nn_conv3d_bwd_weight for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and arguments, with the per-block partial sums in a static device array of
 * 8,388,608 floats (32 MiB, one copy per device, held until the process ends) instead
 * of a buffer allocated per call.  Calls no hipMalloc / hipFree and does not
 * synchronise: the work is enqueued on `stream`.  RT_EINVAL when the layer needs more
 * partial sums than that: 27 * cout * (c1 + c2) floats per block of the weight-gradient
 * grid (min(256, number of 32 x 2 x 2-cell tiles) blocks), and ceil(n / 2048) * cout for
 * the bias; so every layer with cout * (c1 + c2) <= 1024 (16 x 16 ... 16 x 48, 32 x 32)
 * fits at any grid size up to 268 M cells, wider ones only on grids of fewer tiles
 * (64 x 64: at most 75).  Every call on a device shares that device's array: calls that
 * overlap on one device (different streams without ordering, several host threads) race
 * and must be serialised by the caller. */
rt_status rt_nn_conv3d_bwd_weight_noalloc(void *stream, int nr, int nt, int np, const float *dy, const void *yrelu,
                                          int cout, const void *x1, int c1, int up1, const void *x2, int c2, float *dw,
                                          float *db);

#ifdef __cplusplus
}
#endif
#endif /* RTMI_RT_H */
