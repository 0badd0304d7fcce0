"""Benchmark of the radiation step on one MI355X.

A step is one pass of the main loop (ray trace, E^n, FLD assembly, implicit solve to
a relative residual of 1e-8, Newton temperature update, radiative force) on the
512x256x512-cell, 64-bin workload (tau550 = 100 with lognormal clumps, seed 5000,
dt = 1e9 s).  Every timed step starts from the same prepared state (the temperature
in equilibrium with the stellar irradiation and E = a T_bc^4), so the K timed steps do
identical work.  The headline solve mode is timed first (K steps after W warm-up
steps), then the other modes for comparison (at most 3 steps after 1 warm-up step
each).  The headline mode also runs --successive N steps with the
temperature carried over, reported per step (seconds and iterations) under
"successive_steps" (default 50, the 50 coupled steps of the full-scale configuration):
the system gets harder as the radiation field evolves.  Every
mode's answer is checked against the oracle on the whole grid ("oracle_check": the
oracle's own assembly and residual of the GPU's E, the oracle's Newton temperature from
it).  Unless --no-main-loop, the main loop is also run to equilibrium (the run table's
gray / frequency-dependent runs with and without diffusion) on a 2-D disk, reported
under "main_iteration".  The CPU baseline times the oracle on one core (a phi-slab) and
on all cores (the whole grid, OpenMP build of the same source).

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "FLD solve s/step @1e-8 resid, plain FP64 vs learned-precond; ray-trace Gcell·ν/s"
PEAK_HBM_GBS = 8000.0
# Algorithmic bytes per cell of one launch of each solver kernel (see the kernel comments):
# dir: read r, p_old and the three off-diagonals, write p and q; upd: read y, p, r, q, write y, r.
# Red-black reduced modes (-rb), per cell of the full grid: the red pass reads p's two
# inputs at the black cells and every face coefficient once, writes p at the black cells
# and t at the red cells (20 / 40 B); the black pass reads p, t and every face
# coefficient once and writes q (18 / 36 B); the update streams six half-size arrays.
# A multigrid-preconditioned CG iteration (fp64-mg), algorithmic bytes per cell of the
# finest level.  There: the cycle's float32 kernels (pre-sweep 40: r, im, ap, g, dp out
# and back, cp, q, x out; restriction 29: r, x, w, three couplings, 1/4 of a coarse
# write; residual with the prolonged correction 37: r, x, w, 1/4 of the coarse result,
# three couplings, rhs and x' out; last sweep 60: rhs, im, ap, g, dp out and back, cp, q,
# x', r, q_old, z out) and the float64 direction (56) and update (48) kernels: 270.  A
# cycle on a coarser level moves ~142 bytes per cell of that level (its couplings and
# diagonal, float32 right-hand side); levels 1 to 3 take K-cycle steps (two cycles and
# two flexible-CG steps of 96 bytes per cell on level 1; four cycles and two step pairs
# on level 2; eight cycles and four step pairs on level 3; the levels below are visited
# eight times): 95, 48, 24 and ~6 bytes per finest-level cell.
MG_ITER_BYTES_PER_CELL = 270 + 95 + 48 + 24 + 6
# The float32 flexible-CG variant (mixed-mg): the same cycle on a float32 residual (4
# bytes less in each of the first three kernels, the last sweep writes a float32 z and
# reads no r: 40), flexible-CG beta 8 (z, q), direction 32 (three couplings, z, p_old,
# r; p and q out), update 24 (x, p, r, q; x and r out).
MG32_ITER_BYTES_PER_CELL = 36 + 25 + 33 + 40 + 8 + 32 + 24 + 95 + 48 + 24 + 6
# The plain V-cycle (fp64-mgv): the finest level as above, the coarser levels once
# each (~50).
MGV_ITER_BYTES_PER_CELL = 270 + 50
BYTES_PER_CELL = {"fp64": {"dir": 7 * 8, "upd": 6 * 8}, "mixed": {"dir": 7 * 4, "upd": 6 * 4},
                  "fp64-rb": {"dir": 76, "upd": 24, "red": 40, "black": 36},
                  "mixed-rb": {"dir": 38, "upd": 12, "red": 20, "black": 18},
                  "fp64-mg": {"cg_dir": 7 * 8, "upd": 6 * 8, "iteration": MG_ITER_BYTES_PER_CELL},
                  "mixed-mg": {"cg_dir": 32, "upd": 24, "iteration": MG32_ITER_BYTES_PER_CELL},
                  "fp64-mgv": {"cg_dir": 7 * 8, "upd": 6 * 8, "iteration": MGV_ITER_BYTES_PER_CELL}}
KERNEL_NAMES = {"fp64": "k_cg_dir<double>", "mixed": "k_cg_dir<float>", "fp64-rb": ("k_rb_red_dir<double>",
                "k_rb_black_dir<double>"), "mixed-rb": ("k_rb_red_dir<float>", "k_rb_black_dir<float>"),
                "fp64-mg": "k_cg_dir<double>", "mixed-mg": "k_fcg_dir<4>", "fp64-mgv": "k_cg_dir<double>"}
# HBM bytes per launch of these kernels on the 512x256x512 workload, from rocprofv3
# FETCH_SIZE (x2.0, calibrated on a kernel of known size) + WRITE_SIZE; the summary with
# the commands is profiles/solver_kernels_clumpy-512x256x512-nu64.md.  Set to None when
# the kernel changes.
# Keyed by kernel; profiles/rb_solver_kernels_clumpy-512x256x512-nu64.md for the reduced passes.
MEASURED_TRAFFIC = {("k_cg_dir<float>", "clumpy-512x256x512-nu64"): 1.924e9,
                    ("k_cg_dir<double>", "clumpy-512x256x512-nu64"): 3.855e9,
                    ("k_rb_red_dir<float>", "clumpy-512x256x512-nu64"): 1.355e9,
                    ("k_rb_black_dir<float>", "clumpy-512x256x512-nu64"): 1.232e9,
                    ("k_rb_red_dir<double>", "clumpy-512x256x512-nu64"): 2.734e9,
                    ("k_rb_black_dir<double>", "clumpy-512x256x512-nu64"): 2.582e9}


# The ray trace is bound by float64 instruction issue.  On this workload the step's ray
# trace is k_raytrace_r (lanes on radial cells, 8 cells a lane: one VALU instruction of a
# wavefront covers 64 cell-bins, so VALU wave-instructions per cell and bin is a property
# of the kernel; rocprofv3 SQ_INSTS_VALU on the 512x256x512 workload,
# profiles/raytrace_counters_clumpy-512x256x512-nu64.md), and the chip issues at most one
# float64 wave-instruction per CU per cycle (4 SIMDs, 4 cycles per wave64 instruction):
# 256 CUs x 2.4 GHz.  The algorithm itself needs ~35 float64 operations per cell and bin.
# 31.0 is the count where the wavefront's cells all lie below dust sublimation (kappa_nu
# from one table row per bin), as in the benchmark step; 32.9 with the interpolation.
# (Columns that do not fill their 512-cell segments to 90 % take lanes on bins,
# k_raytrace<false, false>, 31.3 instructions per cell and bin.)
RAYTRACE_KERNELS = {True: ("k_raytrace_r", 31.0), False: ("k_raytrace<false, false>", 31.3)}
RAYTRACE_ALG_INSTS_PER_CELL = 35.0


def raytrace_kernel(nr):
    """(kernel name, VALU wave-instructions per cell and bin) of the step's ray trace."""
    seg = -(-nr // 512)
    return RAYTRACE_KERNELS[10 * nr >= 9 * 512 * seg]
PEAK_FP64_WAVE_INSTS = 256 * 2.4e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Multiply-adds x 2 per fine cell of one U-Net application: 3x3x3 layers (Cin x Cout)
# 16x16, 16x16, 48x16, 16x16 on the fine level, 16x32, 32x32, 96x32, 32x32 on the 2x
# coarser level (1/8 of the cells), 32x64, 64x64 on the 4x coarser level (1/64), and
# the 1x1 16 -> 1 output.
UNET_FLOP_PER_CELL = 54 * (256 + 256 + 768 + 256) + 54 * (512 + 1024 + 3072 + 1024) / 8 + 54 * (2048 + 4096) / 64 + 32
PEAK_BF16_TFLOPS = 2500.0


LAUNCH = {"auto": 0, "direct": 1, "graph": 2, "block": 3}  # rt_launch
_launch = 0


def mode_opts(rt, mode, tol, max_iter, inner_tol, net=None, budget=0, restart=30):
    """Solve options of a bench mode; the suffix -rb solves the red-black reduced system,
    -line preconditions float64 CG with the radial-line block Jacobi, -mg with one
    multigrid cycle per iteration (K-cycle steps on levels 1 to 3), -mgv with a plain
    V-cycle; learned-fgmres runs the network inside flexible GMRES(m) instead of
    flexible CG."""
    parts = mode.split("-")
    base = parts[0]
    m = {"fp64": rt.MODE_FP64, "mixed": rt.MODE_MIXED, "learned": rt.MODE_LEARNED, "gmres": rt.MODE_GMRES}[base]
    every = 8 if mode.endswith(("-mg", "-mgv")) else 32  # a multigrid iteration is several passes
    return rt.solve_opts(m, tol=tol, max_iter=max_iter, check_every=every, inner_tol=inner_tol,
                         inner_max_iter=budget if base == "learned" else 0, net=net if base == "learned" else None,
                         restart=restart, reduce=int(mode.endswith("-rb")),
                         precond=1 if mode.endswith("-line") else (2 if mode.endswith(("-mg", "-mgv")) else 0),
                         cycle=rt.CYCLE_V if mode.endswith("-mgv") else rt.CYCLE_K,
                         launch=_launch, inner=rt.INNER_FGMRES if "fgmres" in parts else rt.INNER_FCG)


def train_network(rt, torch, sy, n_fields, epochs, seed=7):
    """The learned preconditioner, trained on the GPU: n_fields seeded clumpy 128x64x64
    fields (tau550 log-uniform in [0.1, 100]), pairs from 0/10/40/150 float64 CG
    iterations, residual loss; then one round of pairs from the learned solver's own
    residuals (1/3/8/20 iterations) and further epochs."""
    import numpy as np
    t0 = time.perf_counter()
    rng = np.random.Generator(np.random.PCG64(seed))
    wls = [sy.make_workload("train", 128, 64, 64, 64, float(10 ** rng.uniform(-1, 2)), 2000 + f)
           for f in range(n_fields)]
    ctx = rt.Context.from_workload(wls[0])
    n = ctx.n

    def system(wl):
        rho = torch.tensor(wl.rho.ravel(), device="cuda")
        T = torch.full((n,), wl.T_bc, dtype=torch.float64, device="cuda")
        q = torch.empty(n, dtype=torch.float64, device="cuda")
        S = torch.empty_like(q)
        ctx.raytrace(rho, T, q, S)
        ctx.temperature(torch.full((n,), sy.A_RAD * wl.T_bc ** 4, dtype=torch.float64, device="cuda"), S, T)
        ctx.raytrace(rho, T, q, S)
        En = torch.empty_like(q)
        ctx.energy(T, S, En)
        ctx.assemble(rho, T, En, q)
        return En

    ds = rt.Dataset(ctx, 8 * n_fields)
    for wl in wls:
        ds.add(system(wl), [0, 10, 40, 150])
    net = rt.Net(seed=seed)
    st0 = net.train(ctx, ds, epochs=epochs, lr=1e-3, seed=1, loss=rt.LOSS_RESIDUAL)
    for wl in wls:
        ds.add_learned(net, system(wl), [1, 3, 8, 20])
    st1 = net.train(ctx, ds, epochs=max(1, epochs // 2), lr=5e-4, seed=2, loss=rt.LOSS_RESIDUAL)
    torch.cuda.synchronize()
    info = {"fields": n_fields, "grid": "128x64x64", "pairs": len(ds), "steps": st0["steps"] + st1["steps"],
            "loss": "residual", "loss_first_epoch": st0["loss_first_epoch"], "loss_last_epoch": st1["loss_last_epoch"],
            "train_s": time.perf_counter() - t0}
    del ds, ctx
    torch.cuda.empty_cache()
    return net, info


def prepared_system(ctx, torch, sy, wl):
    """Assembles the first radiation step's system of workload wl on ctx (irradiation at
    T_bc, Eq. 16 with E = a T_bc^4, then the step's ray trace, E^n and assembly) and
    returns E^n and T^n (device)."""
    n = ctx.n
    rho = torch.tensor(wl.rho.ravel(), device="cuda")
    T = torch.full((n,), wl.T_bc, dtype=torch.float64, device="cuda")
    q = torch.empty(n, dtype=torch.float64, device="cuda")
    S = torch.empty_like(q)
    ctx.raytrace(rho, T, q, S)
    ctx.temperature(torch.full((n,), sy.A_RAD * wl.T_bc ** 4, dtype=torch.float64, device="cuda"), S, T)
    ctx.raytrace(rho, T, q, S)
    En = torch.empty_like(q)
    ctx.energy(T, S, En)
    ctx.assemble(rho, T, En, q)
    return En, T


def c4_gain(rt, torch, sy, n_fields=200, eval_seeds=(10000, 10001, 10002, 10003, 10004), epochs=6,
            fcg_budget=1500):
    """The learned preconditioner's gain as the config states it: trained on n_fields
    seeded clumpy 128x64x64 fields (tau550 log-uniform in [0.1, 100]), evaluated on unseen
    seeds at 256x128x256 (tau550 = 100, 64 bins).  Per evaluation field, iterations and
    seconds to the relative residual 1e-8 of: learned flexible CG (the trained network,
    up to fcg_budget applications before the planned float64 finish), the same with an
    untrained network of the same shape, Jacobi-preconditioned CG (float64; Jacobi FCG is
    CG on the Jacobi-scaled system), the same three with flexible GMRES(30) (the network
    as its right preconditioner; plain GMRES(30) on the Jacobi-scaled system), and the
    benchmark's reduced solves with and without five network applications in front
    (learned-rb vs mixed-rb)."""
    t0 = time.perf_counter()
    net, info = train_network(rt, torch, sy, n_fields, epochs)
    untrained = rt.Net(seed=12345)
    wl0 = sy.make_workload("c4-eval", 256, 128, 256, 64, 100.0, eval_seeds[0])
    ctx = rt.Context.from_workload(wl0)
    rows = []
    FG = rt.INNER_FGMRES
    modes = {"learned_fcg": (rt.MODE_LEARNED, net, fcg_budget, 0, rt.INNER_FCG),
             "untrained_fcg": (rt.MODE_LEARNED, untrained, fcg_budget, 0, rt.INNER_FCG),
             "jacobi_cg_fp64": (rt.MODE_FP64, None, 0, 0, rt.INNER_FCG),
             "learned_fgmres": (rt.MODE_LEARNED, net, fcg_budget, 0, FG),
             "untrained_fgmres": (rt.MODE_LEARNED, untrained, fcg_budget, 0, FG),
             "jacobi_gmres_fp64": (rt.MODE_GMRES, None, 0, 0, rt.INNER_FCG),
             "learned_rb_5": (rt.MODE_LEARNED, net, 5, 1, rt.INNER_FCG),
             "mixed_rb": (rt.MODE_MIXED, None, 0, 1, rt.INNER_FCG)}
    for seed in eval_seeds:
        wl = wl0 if seed == eval_seeds[0] else sy.make_workload("c4-eval", 256, 128, 256, 64, 100.0, seed)
        En, _ = prepared_system(ctx, torch, sy, wl)
        row = {"seed": seed}
        for name, (m, nt, budget, red, inner) in modes.items():
            E = En.clone()
            # plain restarted GMRES on an SPD system can take many times CG's iterations
            o = rt.solve_opts(m, tol=1e-8, max_iter=20000 if m == rt.MODE_GMRES else 200000, net=nt,
                              inner_max_iter=budget, reduce=red, restart=30, inner=inner)
            torch.cuda.synchronize()
            t = time.perf_counter()
            rc, st = ctx.solve(E, o, raise_on_error=False)
            torch.cuda.synchronize()
            row[name] = {"s": time.perf_counter() - t, "iters": st["iters"],
                         "network_applications": st["precond_applies"], "handover": st["handover"],
                         "fallback": st["fallback"], "relres": st["relres"], "status": rc}
            log(f"c4 seed {seed} {name}: {row[name]}")
        rows.append(row)

    def med(name, key):
        return statistics.median([r[name][key] for r in rows])
    summary = {name: {"median_s": med(name, "s"), "median_iters": med(name, "iters"),
                      "median_network_applications": med(name, "network_applications"),
                      "reached_tol_without_handover": sum(1 for r in rows if r[name]["handover"] == 0)}
               for name in modes}
    return {"what": "config 4: network trained on 128x64x64 fields, evaluated on unseen seeds at 256x128x256, "
                    "tau550 = 100, 64 bins; seconds and iterations to relative residual 1e-8",
            "training": info, "fcg_budget": fcg_budget, "eval_seeds": list(eval_seeds), "summary": summary,
            "fields": rows, "total_s": time.perf_counter() - t0}


def unet_forward_ms(ctx, net, torch, reps=3):
    """Average duration of one network application on the context's grid (HIP events on
    the stream the kernels run on): the forward pass on a prepared input (rt_net_forward)
    and the preconditioner's action on a residual as the learned solve applies it
    (rt_net_apply: the scaling reduction, the input built inside the first convolution,
    the forward pass, the output scaled back)."""
    n = ctx.n
    X = (torch.randn(n * 16, device="cuda") * 0.5).to(torch.bfloat16)
    r = torch.randn(n, device="cuda")
    z = torch.empty(n, dtype=torch.float32, device="cuda")
    out = {}
    for name, fn in (("forward", lambda: net.forward(ctx, X, z)), ("apply", lambda: net.apply(ctx, r, z))):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / reps
    del X, r, z
    return out


def run_mode(ctx, rt, torch, rho, T0, mode, steps, warmup, tol, inner_tol, max_iter, net=None, budget=0):
    n = ctx.n
    opts = mode_opts(rt, mode, tol, max_iter, inner_tol, net, budget)
    T = T0.clone()
    E = torch.empty(n, dtype=torch.float64, device="cuda")
    f = torch.empty(4 * n, dtype=torch.float64, device="cuda")
    for w in range(warmup):
        T.copy_(T0)
        rc, st = ctx.step(rho, T, E, opts, f_rad=f)
        log(f"[{mode}] warmup step {w}: solve {st['solve']['ms']:.1f} ms, {st['solve']['iters']} it, "
            f"relres {st['solve']['relres']:.2e}")
    stats = []
    wall = 0.0
    for k in range(steps):
        T.copy_(T0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, st = ctx.step(rho, T, E, opts, f_rad=f)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        stats.append(st)
        log(f"[{mode}] step {k}: total {st['ms_total']:.1f} ms, raytrace {st['ms_raytrace']:.2f} ms, "
            f"solve {st['solve']['ms']:.1f} ms ({st['solve']['iters']} it, {st['solve']['outer_iters']} outer, "
            f"{st['solve']['precond_applies']} network applications, handover {st['solve']['handover']}, "
            f"fallback {st['solve']['fallback']}, "
            f"relres {st['solve']['relres']:.2e}, reduced {st['solve']['reduced']}), "
            f"dir {st['solve']['ms_dir']*1e3:.1f} us, black {st['solve']['ms_black']*1e3:.1f} us, "
            f"upd {st['solve']['ms_upd']*1e3:.1f} us")
    return dict(wall_s=wall, stats=stats, T=T, E=E, f=f)


def run_successive(ctx, rt, torch, rho, T0, mode, nsteps, tol, inner_tol, max_iter, net=None, budget=0):
    """nsteps steps carrying the temperature over; per-step solve statistics."""
    opts = mode_opts(rt, mode, tol, max_iter, inner_tol, net, budget)
    T = T0.clone()
    E = torch.empty(ctx.n, dtype=torch.float64, device="cuda")
    out = []
    for k in range(nsteps):
        rc, st = ctx.step(rho, T, E, opts, raise_on_error=False)
        s = st["solve"]
        out.append({"step": k + 1, "iters": s["iters"], "solve_s": s["ms"] / 1e3, "step_s": st["ms_total"] / 1e3,
                    "relres": s["relres"], "fallback": s["fallback"], "status": rc,
                    "T_max": float(T.max()), "T_mean": float(T.mean())})
        log(f"[{mode}] successive step {k + 1}: solve {s['ms']:.1f} ms, {s['iters']} it, relres {s['relres']:.2e}, "
            f"fallback {s['fallback']}, status {rc}")
    return out


def run_main_loop(rt, torch, sy, shape=(64, 64, 1), n_nu=64, tol_change=1e-4):
    """The run table's main-loop runs on a 2-D disk (the stand-in for the paper's 60x61
    grid): gray (G) or frequency-dependent (F) irradiation, without or with diffusion
    (D), from T_bc at dt = 1e4 s until the largest relative temperature change of a
    step is below tol_change.  Also the gray/frequency-dependent midplane temperature
    ratio of each pair (the analogue of the run table's deviation row)."""
    runs, mid = {}, {}
    for tau, gray, fld in ((0.1, True, False), (100.0, True, False), (100.0, False, False),
                           (100.0, True, True), (100.0, False, True)):
        name = ("G" if gray else "F") + ("D" if fld else "") + f"{tau:g}"
        wl = sy.make_workload("disk-2d", *shape, n_nu, tau, None, dt=1e4)
        ctx = rt.Context.from_workload(wl, gray=gray)
        rho = torch.tensor(wl.rho.ravel(), device="cuda")
        T = torch.full((ctx.n,), wl.T_bc, dtype=torch.float64, device="cuda")
        E = torch.empty_like(T)
        o = rt.solve_opts(rt.MODE_FP64, tol=1e-8, reduce=1) if fld else rt.solve_opts(rt.MODE_NONE)
        t = time.perf_counter()
        rc, st = ctx.relax(rho, T, E, o, tol_change=tol_change, max_steps=5000, raise_on_error=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        runs[name] = {"status": rc, "steps": st["steps"], "last_change": st["last_change"],
                      "krylov_iters": st["krylov_iters"], "s": wall, "ms_per_step": wall / st["steps"] * 1e3}
        j = shape[1] // 2  # the cell row just below the equator
        mid[name] = T.view(shape[2], shape[1], shape[0])[0, j].cpu().numpy()
        if fld:  # Fig. 8: the Rosseland depth through the midplane, inward from r_out
            tau = torch.empty((shape[0] + 1) * shape[1] * shape[2], dtype=torch.float64, device="cuda")
            ctx.rosseland_depth(rho, T, tau)
            runs[name]["tau_R_midplane_r_in"] = float(tau.view(shape[2], shape[1], shape[0] + 1)[0, j, 0])
        log(f"main loop {name}: {runs[name]}")
        del ctx
    cmp = {}
    for g, f in (("G100", "F100"), ("GD100", "FD100")):
        r = mid[g] / mid[f] - 1.0
        cmp[f"{g}_vs_{f}"] = {"max_percent": float(r.max() * 100), "min_percent": float(r.min() * 100)}
    # the GD100 run again with each step launched from the host (the one-workgroup solve
    # per step), and with the iterations launched kernel by kernel and from graphs (the
    # runs above take the default: every step replayed from one captured graph, its solve
    # in one workgroup)
    launch = {"step_graph": {"s": runs["GD100"]["s"], "ms_per_step": runs["GD100"]["ms_per_step"],
                             "us_per_krylov_iter": runs["GD100"]["s"] / runs["GD100"]["krylov_iters"] * 1e6}}
    wl = sy.make_workload("disk-2d", *shape, n_nu, 100.0, None, dt=1e4)
    for name, lv in (("block", rt.LAUNCH_BLOCK), ("direct", rt.LAUNCH_DIRECT), ("graph", rt.LAUNCH_GRAPH)):
        ctx = rt.Context.from_workload(wl, gray=True)
        rho = torch.tensor(wl.rho.ravel(), device="cuda")
        T = torch.full((ctx.n,), wl.T_bc, dtype=torch.float64, device="cuda")
        E = torch.empty_like(T)
        t = time.perf_counter()
        rc, st = ctx.relax(rho, T, E, rt.solve_opts(rt.MODE_FP64, tol=1e-8, reduce=1, launch=lv),
                           tol_change=tol_change, max_steps=5000, raise_on_error=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        launch[name] = {"s": wall, "ms_per_step": wall / max(st["steps"], 1) * 1e3,
                        "us_per_krylov_iter": wall / max(st["krylov_iters"], 1) * 1e6,
                        "steps": st["steps"], "status": rc}
        log(f"main loop GD100, launch {name}: {launch[name]}")
        del ctx
    return {"workload": f"disk-2d {shape[0]}x{shape[1]}x{shape[2]} cells, {n_nu} bins, no clumps, dt=1e4 s, "
                        f"stop when max |dT/T| < {tol_change:g}; FLD solves reduced float64 CG to 1e-8",
            "runs": runs, "gray_vs_freq_midplane": cmp, "gd100_by_launch": launch}


def rosseland_depth_rate(ctx, torch, rho, T, reps=5):
    """Time rt_rosseland_depth (one kernel) on the prepared state: ms per launch, its
    algorithmic bytes (T and rho in, tau_R out at the faces) per second, and the
    midplane tau_R at r_in."""
    nr, nt, npp = ctx.shape
    tau = torch.empty((nr + 1) * nt * npp, dtype=torch.float64, device="cuda")
    ctx.rosseland_depth(rho, T, tau)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        ctx.rosseland_depth(rho, T, tau)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    nbytes = 16 * nr * nt * npp + 8 * (nr + 1) * nt * npp
    gbs = nbytes / (ms / 1e3) / 1e9
    return {"kernel": "k_tau_rosseland", "ms": ms, "achieved_GBs": gbs, "frac_of_8TBs": gbs / PEAK_HBM_GBS,
            "bytes": nbytes, "tau_R_midplane_r_in": float(tau.view(npp, nt, nr + 1)[0, nt // 2, 0])}


def raytrace_mappings(ctx, rt, torch, rho, T, n_nu, reps=5):
    """The step's ray trace with lanes on bins (k_raytrace) against lanes on radial cells
    (k_raytrace_r), both through rt_raytrace_mapped, on the prepared state: mean ms per
    launch over reps launches each (HIP events on the context's stream), the rate, and
    the largest relative difference of their q and S."""
    n = ctx.n
    out = {}
    res = {}
    for name, mapping in (("lanes_bins", rt.LANES_BINS), ("lanes_cells", rt.LANES_CELLS)):
        q = torch.empty(n, dtype=torch.float64, device="cuda")
        S = torch.empty_like(q)
        ctx.raytrace_mapped(mapping, rho, T, q, S)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(reps):
            ctx.raytrace_mapped(mapping, rho, T, q, S)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / reps
        out[name] = {"ms": ms, "gcell_nu_per_s": n * n_nu / (ms / 1e3) / 1e9}
        res[name] = (q, S)
    (q1, S1), (q2, S2) = res["lanes_bins"], res["lanes_cells"]
    relq = ((q2 - q1).abs() / q1.abs().clamp_min(1e-30 * float(q1.abs().max()))).max()
    relS = ((S2 - S1).abs() / S1.abs().clamp_min(1e-30 * float(S1.abs().max()))).max()
    out["kernels"] = {"lanes_bins": "k_raytrace<false, false>", "lanes_cells": "k_raytrace_r"}
    out["q_max_rel_diff"] = float(relq)
    out["S_max_rel_diff"] = float(relS)
    out["cells_over_bins_time"] = out["lanes_cells"]["ms"] / out["lanes_bins"]["ms"]
    out["step_uses"] = "lanes_cells" if raytrace_kernel(ctx.shape[0])[0] == "k_raytrace_r" else "lanes_bins"
    del res, q1, S1, q2, S2
    torch.cuda.empty_cache()
    return out


def _host_info():
    """nproc and the CPU model (lscpu) of the host the baseline ran on."""
    import subprocess
    info = {"nproc": os.cpu_count()}
    try:
        info["nproc"] = int(subprocess.run(["nproc"], capture_output=True, text=True, timeout=10).stdout.strip())
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)",
                             "CPU max MHz"):
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError, ValueError):
        pass
    return info


def oracle_baseline(wl, gpu_fp64_iters, slab=16, cg_iters=1000):
    """The serial oracle (one core) on a phi-slab of the workload: ray trace, Newton,
    assembly and a fixed number of CG iterations, scaled to the full grid and to the GPU
    float64 iteration count."""
    import numpy as np

    import oracle
    from paper_1001_3301_amd import synth as sy
    g = wl.grid
    slab = min(slab, g.shape[2])
    P = oracle.Problem(g.r_face, g.th_face, g.ph_face[: slab + 1], wl.opacity.T, wl.opacity.kappa,
                       wl.opacity.kappa_P, wl.opacity.kappa_R, R_star=wl.R_star,
                       F0=oracle.star_bins(wl.T_star, wl.opacity.nu), dt=wl.dt, c_V=wl.c_V,
                       T_bc=wl.T_bc, E_floor=wl.E_floor)
    rho = np.ascontiguousarray(wl.rho[:slab])
    T = np.full(P.n, wl.T_bc)
    t = time.perf_counter()
    q, S, _ = P.raytrace(rho, T, want_faces=False)
    t_rt = time.perf_counter() - t
    t = time.perf_counter()
    T = P.newton(np.full(P.n, sy.A_RAD * wl.T_bc ** 4), S, T)
    t_nw = time.perf_counter() - t
    En = P.energy(T, S)
    t = time.perf_counter()
    sysd = P.assemble(rho, T, En, q)
    t_as = time.perf_counter() - t
    t = time.perf_counter()
    _, _, it, _ = P.cg(sysd["ahat"], sysd["bhat"], En / sysd["s"], 1e-30, cg_iters)
    t_cg = time.perf_counter() - t
    scale = g.ncell / P.n
    per_iter_full = t_cg / max(it, 1) * scale
    return dict(solve_s_per_step=per_iter_full * gpu_fp64_iters,
                raytrace_gcell_nu=P.n * wl.opacity.kappa.shape[1] / t_rt / 1e9,
                phases_s_full_grid={"raytrace": t_rt * scale, "assemble": t_as * scale, "newton": t_nw * scale,
                                    "cg_iteration": per_iter_full},
                sample=f"serial oracle on a {g.shape[0]}x{g.shape[1]}x{slab} phi-slab of the workload "
                       f"({P.n} cells, 1/{scale:.0f} of the grid): one ray trace ({t_rt:.1f} s) and "
                       f"{it} float64 CG iterations ({t_cg:.1f} s); solve s/step = time per iteration "
                       f"x {scale:.0f} x the GPU float64 iteration count ({gpu_fp64_iters})")


def oracle_full_grid(wl, cg_iters=40):
    """The OpenMP oracle on all host cores, whole grid: its own prepared state (ray trace
    at T_bc, Newton with E = a T_bc^4), the step's ray trace, E^n and assembly, and
    cg_iters float64 CG iterations, each phase timed.  Returns the oracle problem, its
    state and the timings."""
    import numpy as np

    import oracle
    from paper_1001_3301_amd import synth as sy
    P = oracle.Problem.from_workload(wl, parallel=True)
    rho = wl.rho.ravel()
    tm = {}
    t = time.perf_counter()
    _, S, _ = P.raytrace(rho, np.full(P.n, wl.T_bc), want_faces=False)
    tm["raytrace"] = time.perf_counter() - t
    t = time.perf_counter()
    T0 = P.newton(np.full(P.n, sy.A_RAD * wl.T_bc ** 4), S, np.full(P.n, wl.T_bc))
    tm["newton"] = time.perf_counter() - t
    q, S, _ = P.raytrace(rho, T0, want_faces=False)
    En = P.energy(T0, S)
    t = time.perf_counter()
    sysd = P.assemble(rho, T0, En, q)
    tm["assemble"] = time.perf_counter() - t
    for k in ("w", "d", "b"):
        del sysd[k]
    t = time.perf_counter()
    _, _, it, _ = P.cg(sysd["ahat"], sysd["bhat"], En / sysd["s"], 1e-30, cg_iters)
    tm["cg_iteration"] = (time.perf_counter() - t) / max(it, 1)
    return P, dict(T0=T0, S=S, q=q, En=En, **sysd), tm, oracle.threads()


def oracle_check(P, O, E, T):
    """The oracle's residual of the GPU's E on the oracle's own assembled system, and the
    largest relative difference between the GPU's temperature and the oracle's Newton
    step from that E (with the oracle's S and T^n), over every cell."""
    import numpy as np
    Eg = E.cpu().numpy()
    res = P.relres(O["ahat"], O["bhat"], Eg / O["s"])
    Tn = P.newton(Eg, O["S"], O["T0"])
    Tg = T.cpu().numpy()
    return {"oracle_relres": float(res), "T_vs_oracle_newton_max_rel": float(np.max(np.abs(Tg - Tn) / Tn))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="clumpy-512x256x512-nu64")
    ap.add_argument("--modes", default="fp64-mg,fp64-mgv,mixed-rb,fp64,mixed,fp64-rb,learned,learned-rb,"
                                       "learned-fgmres-rb",
                    help="comma list; the first is the headline (suffix -rb: red-black reduced system)")
    ap.add_argument("--net", default="", help="load the network from this file instead of training it")
    ap.add_argument("--save-net", default="", help="save the trained network to this file")
    ap.add_argument("--train-fields", type=int, default=24)
    ap.add_argument("--train-epochs", type=int, default=6)
    ap.add_argument("--learned-budget", type=int, default=50,
                    help="network applications before the learned solve hands over to float64 CG")
    ap.add_argument("--learned-rb-budget", type=int, default=5,
                    help="the same for learned-rb, which hands over to the reduced mixed solve")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--inner-tol", type=float, default=1e-4)
    ap.add_argument("--max-iter", type=int, default=200000)
    ap.add_argument("--successive", type=int, default=50,
                    help="also run this many successive steps of the headline mode (not timed for value; "
                         "50 x ~0.5 s with the multigrid headline, far longer with a Jacobi-CG headline)")
    ap.add_argument("--successive-also", default="fp64-mgv",
                    help="comma list of further modes that also run the successive steps")
    ap.add_argument("--other-steps", type=int, default=3,
                    help="timed steps of each non-headline mode (at most --steps; warm-up at most 1)")
    ap.add_argument("--c4-gain", action="store_true",
                    help="run only the config-4 gain evaluation (200 training fields at 128x64x64, unseen "
                         "256x128x256 seeds) and print its JSON")
    ap.add_argument("--c4-fields", type=int, default=200)
    ap.add_argument("--no-oracle-check", action="store_true",
                    help="skip the whole-grid oracle check of every mode's answer")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-main-loop", action="store_true", help="skip the main-loop runs to equilibrium")
    ap.add_argument("--launch", choices=list(LAUNCH), default="auto",
                    help="how the solver's iterations are launched (rt_launch); kernel times are sampled "
                         "only with direct launches, which auto takes above 4,194,304 cells")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="copy a buffer of this size once before timing (HBM-counter calibration)")
    args = ap.parse_args()
    global _launch
    _launch = LAUNCH[args.launch]
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the radiation step runs on a single MI355X; "
              "splitting it over several GPUs (phi-slabs with halo planes) is designed, not implemented",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1001_3301_amd import rt, synth as sy
    torch.cuda.set_device(0)
    if args.c4_gain:
        print(json.dumps(c4_gain(rt, torch, sy, n_fields=args.c4_fields, epochs=args.train_epochs)), flush=True)
        return
    t = time.perf_counter()
    c = sy.CONFIGS[args.config]
    wl = sy.make_workload(args.config, c["nr"], c["nt"], c["nph"], c["n_nu"], c["taus"][-1],
                          c["seeds"][-1])
    log(f"workload {args.config}: {wl.grid.shape}, {c['n_nu']} bins, tau550={wl.tau550}, "
        f"generated in {time.perf_counter() - t:.1f} s")
    ctx = rt.Context.from_workload(wl)
    n = ctx.n
    rho = torch.tensor(wl.rho.ravel(), device="cuda")
    # initial temperature: irradiation at T_bc, then Eq. 16 with E = a T_bc^4 (all on the GPU)
    T0 = torch.full((n,), wl.T_bc, dtype=torch.float64, device="cuda")
    q = torch.empty(n, dtype=torch.float64, device="cuda")
    S = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.raytrace(rho, T0, q, S)
    E0 = torch.full((n,), sy.A_RAD * wl.T_bc ** 4, dtype=torch.float64, device="cuda")
    ctx.temperature(E0, S, T0)
    del q, S, E0
    torch.cuda.synchronize()

    if args.calib_copy_mib > 0:
        src = torch.ones(args.calib_copy_mib * 2 ** 20 // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"calibration copy of {args.calib_copy_mib} MiB done")

    modes = [m.strip() for m in args.modes.split(",") if m.strip()]
    net, train_info = None, None
    learned_modes = [m for m in modes if m.startswith("learned")]
    if learned_modes:
        if args.net:
            net = rt.Net(seed=1)
            net.load(args.net)
            train_info = {"loaded": args.net}
        else:
            net, train_info = train_network(rt, torch, sy, args.train_fields, args.train_epochs)
            if args.save_net:
                net.save(args.save_net)
        log(f"network: {train_info}")
    results = {}
    for mi, mode in enumerate(modes):
        budget = args.learned_rb_budget if mode.startswith("learned") and mode.endswith("-rb") else args.learned_budget
        steps = args.steps if mi == 0 else min(args.steps, args.other_steps)
        warm = args.warmup if mi == 0 else min(args.warmup, 1)
        results[mode] = run_mode(ctx, rt, torch, rho, T0, mode, steps, warm, args.tol,
                                 args.inner_tol, args.max_iter, net, budget)

    head = modes[0]
    R = results[head]
    solve_s = [s["solve"]["ms"] / 1e3 for s in R["stats"]]
    rt_ms = [s["ms_raytrace"] for s in R["stats"]]
    value = statistics.median(solve_s)
    samples = sum(s["solve"]["kernel_samples"] for s in R["stats"])
    ms_dir = sum(s["solve"]["ms_dir"] * s["solve"]["kernel_samples"] for s in R["stats"]) / max(samples, 1)
    ms_upd = sum(s["solve"]["ms_upd"] * s["solve"]["kernel_samples"] for s in R["stats"]) / max(samples, 1)
    ms_black = sum(s["solve"]["ms_black"] * s["solve"]["kernel_samples"] for s in R["stats"]) / max(samples, 1)
    bpc = BYTES_PER_CELL.get(head)
    # the dominant kernel: the direction kernel, or the longer of the red and black passes
    # of a reduced solve (bytes per half-grid cell = twice the per-full-cell figure)
    kname = KERNEL_NAMES.get(head)
    if bpc and "iteration" in bpc:
        # multigrid CG: the float64 direction kernel is the longest launch of an iteration
        # (ms_black times it alone; ms_dir - ms_black is the V-cycle)
        dom_b, dom_ms, dom_cells = bpc["cg_dir"], ms_black, n
    elif bpc and "black" in bpc:
        ms_red = ms_dir - ms_black
        red_dom = ms_red > ms_black
        dom_b, dom_ms, dom_cells = (2 * bpc["red"], ms_red, n // 2) if red_dom else (2 * bpc["black"], ms_black, n // 2)
        kname = kname[0] if red_dom else kname[1]
    else:
        dom_b, dom_ms, dom_cells = (bpc["dir"], ms_dir, n) if bpc else (0, 0.0, n)
    achieved = dom_b * dom_cells / (dom_ms / 1e3) / 1e9 if (bpc and dom_ms > 0) else 0.0
    rt_kernel, rt_valu = raytrace_kernel(ctx.shape[0])
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "s/step",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": R["wall_s"] / args.steps * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f64+f32" if head.startswith("fp64") else "f32+f64") if head.endswith(("-mg", "-mgv")) else
                 {"fp64": "f64", "mixed": "f32+f64", "learned": "bf16+f32+f64", "gmres": "f64"}[head.split("-")[0]],
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {wl.grid.shape[0]}x{wl.grid.shape[1]}x{wl.grid.shape[2]} cells, "
                               f"{c['n_nu']} bins, tau550={wl.tau550:g}, clumps seed {c['seeds'][-1]}",
                   "solve_mode": head, "tol": args.tol, "dt": wl.dt,
                   "step": "first step from the prepared state, repeated K times"},
        "raytrace_gcell_nu_per_s": statistics.median([n * c["n_nu"] / (x / 1e3) / 1e9 for x in rt_ms]),
        "raytrace_roofline": {"kernel": rt_kernel, "bound": "alu",
                              "unit": "float64 VALU wave-instructions/s",
                              "achieved": rt_valu * n / (statistics.median(rt_ms) / 1e3),
                              "peak": PEAK_FP64_WAVE_INSTS,
                              "frac": rt_valu * n / (statistics.median(rt_ms) / 1e3) / PEAK_FP64_WAVE_INSTS,
                              "valu_insts_per_cell": rt_valu,
                              # the same bound priced on the algorithm's own count rather
                              # than the instructions issued: one exp/expm1 pair and ~8 more
                              # float64 operations per cell-bin, ~35 instructions
                              "algorithmic_insts_per_cell": RAYTRACE_ALG_INSTS_PER_CELL,
                              "algorithmic_frac": RAYTRACE_ALG_INSTS_PER_CELL * n / (statistics.median(rt_ms) / 1e3)
                              / PEAK_FP64_WAVE_INSTS},
        "solve_iters_per_step": statistics.median([s["solve"]["iters"] for s in R["stats"]]),
        "kernel_ms": {"dir": ms_dir, "upd": ms_upd, "black": ms_black, "samples": samples},
    }
    if bpc:
        out["roofline"] = {"kernel": kname, "bound": "hbm", "achieved": achieved,
                           "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                           "traffic": MEASURED_TRAFFIC.get((kname, args.config)), "bytes_per_cell": dom_b,
                           "cells_per_launch": dom_cells}
        if ms_dir > 0 and ms_upd > 0:
            # one whole Krylov iteration (all its kernels): its algorithmic bytes over the launch times
            it_b = bpc["iteration"] if "iteration" in bpc else bpc["dir"] + bpc["upd"]
            it_gbs = it_b * n / ((ms_dir + ms_upd) / 1e3) / 1e9
            out["krylov_iteration"] = {"achieved": it_gbs, "unit": "GB/s", "frac": it_gbs / PEAK_HBM_GBS,
                                       "bytes_per_cell": it_b, "ms": ms_dir + ms_upd}
    for mode in modes[1:]:
        Rm = results[mode]
        out[f"{mode}_solve_s_per_step"] = statistics.median([s["solve"]["ms"] / 1e3 for s in Rm["stats"]])
        out[f"{mode}_iters_per_step"] = statistics.median([s["solve"]["iters"] for s in Rm["stats"]])
    if learned_modes:
        lm = learned_modes[0]
        Rl = results[lm]["stats"][-1]["solve"]
        tm = unet_forward_ms(ctx, net, torch)
        fwd_ms = tm["forward"]
        tflops = UNET_FLOP_PER_CELL * n / (fwd_ms / 1e3) / 1e12
        out["learned"] = {"mode": lm, "network_applications": Rl["precond_applies"], "fallback": Rl["fallback"],
                          "handover": Rl["handover"],
                          "total_iters": Rl["iters"],
                          "budget": args.learned_rb_budget if lm.endswith("-rb") else args.learned_budget,
                          "training": train_info, "unet_forward_ms": fwd_ms, "unet_apply_ms": tm["apply"],
                          "unet_roofline": {"kernel": "U-Net forward (k_conv_fwd and pooling, whole network)",
                                            "bound": "mfma", "achieved": tflops, "peak": PEAK_BF16_TFLOPS,
                                            "unit": "TFLOP/s", "frac": tflops / PEAK_BF16_TFLOPS,
                                            "flop_per_cell": UNET_FLOP_PER_CELL, "cells": n}}
        for m in learned_modes[1:]:
            Rm = results[m]["stats"][-1]["solve"]
            out["learned"][m] = {"network_applications": Rm["precond_applies"], "total_iters": Rm["iters"],
                                 "reduced_finish": Rm["reduced"], "handover": Rm["handover"],
                                 "fallback": Rm["fallback"]}
        if head.startswith("learned"):  # the network is the part of this mode the GPU is asked to run fast
            out["roofline"] = dict(out["learned"]["unet_roofline"], traffic=None)
    if "fp64" in modes:
        Tf, Ef, ff = results["fp64"]["T"], results["fp64"]["E"], results["fp64"]["f"].view(4, -1)
        thermal = ff[1:].norm(dim=0).max()  # the thermal force differentiates E: judged on its scale
        for mode in modes:
            if mode != "fp64":
                Rm = results[mode]
                out[f"T_rel_diff_{mode}_vs_fp64"] = float(((Rm["T"] - Tf).abs() / Tf).max())
                out[f"E_rel_diff_{mode}_vs_fp64"] = float(((Rm["E"] - Ef).abs() / Ef.abs()).max())
                out[f"thermal_force_diff_{mode}_vs_fp64"] = float(
                    (Rm["f"].view(4, -1)[1:] - ff[1:]).abs().max() / thermal)
    out["rosseland_depth"] = rosseland_depth_rate(ctx, torch, rho, T0)
    out["raytrace_mappings"] = raytrace_mappings(ctx, rt, torch, rho, T0, c["n_nu"])
    log(f"ray trace mappings: {out['raytrace_mappings']}")
    full = None
    if not args.no_oracle_check or not args.no_cpu_baseline:
        t = time.perf_counter()
        full = oracle_full_grid(wl)
        log(f"oracle on the whole grid ({full[3]} threads): {full[2]}, {time.perf_counter() - t:.1f} s")
    if not args.no_oracle_check:
        P, O = full[0], full[1]
        chk = {"what": "the oracle's own prepared state and assembled system (OpenMP build, whole grid); for each "
                       "mode the oracle's relative residual of the GPU's E and the largest relative difference "
                       "between the GPU's temperature and the oracle's Newton step from that E",
               "prepared_T_max_rel": float(np.max(np.abs(T0.cpu().numpy() - O["T0"]) / O["T0"]))}
        for mode in modes:
            chk[mode] = oracle_check(P, O, results[mode]["E"], results[mode]["T"])
            log(f"oracle check {mode}: {chk[mode]}")
        out["oracle_check"] = chk
    for mode in modes:
        del results[mode]["T"], results[mode]["E"], results[mode]["f"]
    if args.successive > 0:
        also = [m.strip() for m in args.successive_also.split(",") if m.strip() and m.strip() != head]
        for k, smode in enumerate([head] + also):
            seq = run_successive(ctx, rt, torch, rho, T0, smode, args.successive, args.tol, args.inner_tol,
                                 args.max_iter, net, args.learned_budget)
            key = "successive_steps" if k == 0 else f"successive_steps_{smode}"
            out[key] = {
                "what": f"{args.successive} successive radiation steps of the {'headline ' if k == 0 else ''}mode "
                        f"{smode} at dt = {wl.dt:g} s, each from the previous step's temperature (the timed steps "
                        f"above all repeat step 1); solve seconds and iterations per step",
                "mode": smode, "steps": seq, "solve_s_total": sum(x["solve_s"] for x in seq),
                "iters": [x["iters"] for x in seq]}
    if not args.no_main_loop:
        out["main_iteration"] = run_main_loop(rt, torch, sy)
    if not args.no_cpu_baseline:
        fp64_iters = out.get("fp64_iters_per_step", out["solve_iters_per_step"])
        t = time.perf_counter()
        cb = oracle_baseline(wl, fp64_iters)
        log(f"cpu baseline (one core) took {time.perf_counter() - t:.1f} s")
        tm, thr = full[2], full[3]
        host = _host_info()
        out["cpu_baseline"] = {
            "value": tm["cg_iteration"] * fp64_iters, "unit": "s/step", "cores": thr, "kind": "oracle",
            "sample": f"OpenMP oracle on {thr} threads, whole {wl.grid.shape[0]}x{wl.grid.shape[1]}x"
                      f"{wl.grid.shape[2]} grid: ray trace, Newton, assembly and 40 float64 CG iterations; "
                      f"solve s/step = time per CG iteration x the GPU float64 iteration count ({fp64_iters}), "
                      f"the plain method (the oracle has no reduced, mixed-precision or multigrid solve)",
            "phases_s": {"raytrace": tm["raytrace"], "newton": tm["newton"], "assemble": tm["assemble"],
                         "cg_iteration": tm["cg_iteration"]},
            "raytrace_gcell_nu_per_s": n * c["n_nu"] / tm["raytrace"] / 1e9,
            "host": host,
            "single_core": {"value": cb["solve_s_per_step"], "unit": "s/step", "cores": 1, "sample": cb["sample"],
                            "raytrace_gcell_nu_per_s": cb["raytrace_gcell_nu"],
                            "phases_s_full_grid": cb["phases_s_full_grid"]}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
