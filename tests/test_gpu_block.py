"""The one-workgroup reduced float64 CG (rt_solve_opts.launch = RT_LAUNCH_BLOCK, the
default for reduced float64 solves of at most 2048 black cells).

It solves the same system as the multi-block kernels with the dot products summed in
another order, so it is checked against the oracle's dense Cholesky solve of the full
system (grids the dense solve takes) and against the multi-block solve and the
full-system residual recomputed by rt_spmv (grids at the 2048-black-cell limit: two
cells for every thread), and for bitwise repeatability.
"""
import numpy as np
import pytest

import oracle
from paper_1001_3301_amd import synth as sy
from _util import rel, initial_temperature

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _d(x):
    return torch.tensor(np.ascontiguousarray(x, dtype=np.float64).ravel(), device="cuda")


def _h(t):
    return t.detach().cpu().numpy()


def _system(wl):
    from paper_1001_3301_amd import rt
    P = oracle.Problem.from_workload(wl)
    ctx = rt.Context.from_workload(wl)
    T = initial_temperature(P, wl)
    q, S, _ = P.raytrace(wl.rho, T, want_faces=False)
    En = P.energy(T, S)
    ref = P.assemble(wl.rho, T, En, q)
    ctx.assemble(_d(wl.rho), _d(T), _d(En), _d(q))
    return P, ctx, T, S, En, ref


def _full_relres(ctx, E, s, bhat):
    y = E / s
    Ay = torch.empty_like(y)
    ctx.spmv(y, Ay)
    return float(torch.linalg.vector_norm(bhat - Ay) / torch.linalg.vector_norm(bhat))


def _solve(ctx, En, launch, tol, max_iter=100000):
    from paper_1001_3301_amd import rt
    E = _d(En)
    rc, st = ctx.solve(E, rt.solve_opts(rt.MODE_FP64, tol=tol, max_iter=max_iter, reduce=1, launch=launch),
                       raise_on_error=False)
    torch.cuda.synchronize()
    return rc, st, E


DENSE = {  # the oracle's dense solve takes up to 4096 cells
    "axisym-64x16x1": lambda: sy.make_workload("a", 64, 16, 1, 32, 1.0),
    "thick-40x9x4": lambda: sy.make_workload("t", 40, 9, 4, 64, 100.0, clump_seed=3),
    "one-theta-row-16x1x8": lambda: sy.make_workload("o", 16, 1, 8, 8, 10.0, clump_seed=9),
    "two-phi-20x6x2": lambda: sy.make_workload("p", 20, 6, 2, 8, 10.0, clump_seed=10),
    "disk-2d-60x61x1": lambda: sy.make_workload("disk-2d", 60, 61, 1, 16, 100.0, None, dt=1e4),  # the paper's grid size: 2 cells per thread
}

LARGE = {  # the 2048-black-cell limit: every thread owns two cells
    "disk-2d-64x64x1": lambda: sy.make_workload("disk-2d", 64, 64, 1, 16, 100.0, None, dt=1e4),
    "clumpy-32x16x8": lambda: sy.make_workload("c", 32, 16, 8, 8, 10.0, clump_seed=12),
}


@pytest.mark.parametrize("case", list(DENSE))
def test_block_solve_against_dense_oracle(case):
    from paper_1001_3301_amd import rt
    wl = DENSE[case]()
    P, ctx, T, S, En, ref = _system(wl)
    yd = P.dense_solve(ref["ahat"], ref["bhat"])
    rc, st, E = _solve(ctx, En, rt.LAUNCH_BLOCK, 1e-13)
    assert rc == 0 and st["reduced"] == 1 and st["relres"] <= 1e-13
    y = _h(E) / ref["s"]
    assert P.relres(ref["ahat"], ref["bhat"], y) <= 2e-13
    assert rel(y, yd) < 1e-8
    assert _full_relres(ctx, E, _d(ref["s"]), _d(ref["bhat"])) <= 2e-13
    assert rel(P.newton(_h(E), S, T), P.newton(yd * ref["s"], S, T)) < 1e-11
    # the multi-block kernels: the same iteration count up to rounding of the sums
    rc2, st2, E2 = _solve(ctx, En, rt.LAUNCH_DIRECT, 1e-13)
    assert abs(st["iters"] - st2["iters"]) <= max(2, 0.02 * st2["iters"]), (st["iters"], st2["iters"])


@pytest.mark.parametrize("case", list(LARGE))
def test_block_solve_against_multiblock(case):
    from paper_1001_3301_amd import rt
    wl = LARGE[case]()
    P, ctx, T, S, En, ref = _system(wl)
    nh = P.n // 2
    assert nh == 2048
    rc, st, E = _solve(ctx, En, rt.LAUNCH_BLOCK, 1e-12)
    rc2, st2, E2 = _solve(ctx, En, rt.LAUNCH_DIRECT, 1e-12)
    assert rc == rc2 == 0 and st["relres"] <= 1e-12 and st2["relres"] <= 1e-12
    s, b = _d(ref["s"]), _d(ref["bhat"])
    assert _full_relres(ctx, E, s, b) <= 2e-12
    assert rel(_h(E) / ref["s"], _h(E2) / ref["s"]) < 1e-7
    assert rel(P.newton(_h(E), S, T), P.newton(_h(E2), S, T)) < 1e-9
    assert abs(st["iters"] - st2["iters"]) <= max(2, 0.02 * st2["iters"]), (st["iters"], st2["iters"])


def test_block_solve_bitwise_repeatable_and_auto_default():
    """A fixed summation order: two solves give the same bits; RT_LAUNCH_AUTO takes the
    one-workgroup path on this grid (the same bits again)."""
    from paper_1001_3301_amd import rt
    wl = DENSE["disk-2d-60x61x1"]()
    P, ctx, T, S, En, ref = _system(wl)
    outs = [_solve(ctx, En, launch, 1e-12) for launch in (rt.LAUNCH_BLOCK, rt.LAUNCH_BLOCK, rt.LAUNCH_AUTO)]
    for rc, st, E in outs[1:]:
        assert st["iters"] == outs[0][1]["iters"] and np.array_equal(_h(E), _h(outs[0][2]))


def test_block_solve_iteration_limit():
    """max_iter ends the one-workgroup solve exactly there, without convergence."""
    from paper_1001_3301_amd import rt
    wl = DENSE["thick-40x9x4"]()
    P, ctx, T, S, En, ref = _system(wl)
    rc, st, E = _solve(ctx, En, rt.LAUNCH_BLOCK, 1e-14, max_iter=45)
    assert rc == rt.RT_ENOCONV and st["iters"] == 45 and np.all(np.isfinite(_h(E)))


def test_block_too_large_grid_runs_multiblock():
    """Above 2048 black cells RT_LAUNCH_BLOCK falls back to the multi-block kernels
    (the same bits as RT_LAUNCH_GRAPH)."""
    from paper_1001_3301_amd import rt
    wl = sy.make_workload("disk-2d", 66, 64, 1, 8, 100.0, None, dt=1e4)
    P, ctx, T, S, En, ref = _system(wl)
    assert P.n // 2 > 2048
    a = _solve(ctx, En, rt.LAUNCH_BLOCK, 1e-10)
    b = _solve(ctx, En, rt.LAUNCH_GRAPH, 1e-10)
    assert a[1]["iters"] == b[1]["iters"] and np.array_equal(_h(a[2]), _h(b[2]))


def test_relax_with_block_solve_matches_multiblock():
    """The main loop on a 2-D disk with the one-workgroup solve: the same number of main
    iterations and temperatures within the solver tolerance of the multi-block run."""
    from paper_1001_3301_amd import rt
    wl = sy.make_workload("disk-2d", 32, 32, 1, 16, 100.0, None, dt=1e4)
    out = []
    for launch in (rt.LAUNCH_BLOCK, rt.LAUNCH_DIRECT):
        ctx = rt.Context.from_workload(wl, gray=True)
        rho = _d(wl.rho)
        T = torch.full((ctx.n,), wl.T_bc, dtype=torch.float64, device="cuda")
        E = torch.empty_like(T)
        rc, st = ctx.relax(rho, T, E, rt.solve_opts(rt.MODE_FP64, tol=1e-10, reduce=1, launch=launch),
                           tol_change=1e-4, max_steps=2000)
        out.append((st, _h(T)))
    assert out[0][0]["steps"] == out[1][0]["steps"]
    assert rel(out[0][1], out[1][1]) < 1e-6


def test_launch_value_is_checked():
    from paper_1001_3301_amd import rt
    wl = DENSE["thick-40x9x4"]()
    P, ctx, T, S, En, ref = _system(wl)
    for bad in (-1, 4):
        rc, st, E = _solve(ctx, En, bad, 1e-10)
        assert rc == rt.RT_EINVAL
