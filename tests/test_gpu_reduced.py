"""The red-black reduced solve (rt_solve_opts.reduce = 1) against the oracle.

Eliminating the red cells is exact algebra, so the reduced solve must reach the same
solution as the full system: it is checked against the oracle's dense Cholesky solve of
the full system, through the oracle's own residual of the GPU answer, and through the
full-system residual recomputed on the GPU (rt_spmv), on grids with N_phi = 1, even
N_phi, ragged radial rows and a single polar row; grids it cannot colour (odd N_r or
odd N_phi > 1) must fall back to the full system.
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


CASES = {
    "axisym-64x16x1": lambda: sy.make_workload("a", 64, 16, 1, 32, 1.0),
    "thick-40x9x4": lambda: sy.make_workload("t", 40, 9, 4, 64, 100.0, clump_seed=3),
    "clumpy-34x12x6": lambda: sy.make_workload("c", 34, 12, 6, 16, 10.0, clump_seed=8),   # H = 17: one-cell segments
    "one-theta-row-16x1x8": lambda: sy.make_workload("o", 16, 1, 8, 8, 10.0, clump_seed=9),
    "two-phi-20x6x2": lambda: sy.make_workload("p", 20, 6, 2, 8, 10.0, clump_seed=10),  # both phi faces join the same pair
}


@pytest.mark.parametrize("case", list(CASES))
def test_reduced_fp64_solve_against_dense_oracle(case):
    from paper_1001_3301_amd import rt
    wl = CASES[case]()
    P, ctx, T, S, En, ref = _system(wl)
    yd = P.dense_solve(ref["ahat"], ref["bhat"])
    E = _d(En)
    rc, st = ctx.solve(E, rt.solve_opts(rt.MODE_FP64, tol=1e-13, max_iter=20000, check_every=8, reduce=1))
    assert st["reduced"] == 1 and st["relres"] <= 1e-13
    y = _h(E) / ref["s"]
    # the oracle's residual of the recovered full solution (red cells included)
    assert P.relres(ref["ahat"], ref["bhat"], y) <= 2e-13
    assert rel(y, yd) < 1e-8
    assert _full_relres(ctx, E, _d(ref["s"]), _d(ref["bhat"])) <= 2e-13
    Td, Tg = P.newton(yd * ref["s"], S, T), P.newton(_h(E), S, T)
    assert rel(Tg, Td) < 1e-11
    # about half the iterations of the full system at the same tolerance
    E2 = _d(En)
    rc, st2 = ctx.solve(E2, rt.solve_opts(rt.MODE_FP64, tol=1e-13, max_iter=20000, check_every=8))
    assert st2["reduced"] == 0
    assert st["iters"] <= 0.75 * st2["iters"], (st["iters"], st2["iters"])


@pytest.mark.parametrize("case", ["axisym-64x16x1", "thick-40x9x4"])
def test_reduced_mixed_solve(case):
    from paper_1001_3301_amd import rt
    wl = CASES[case]()
    P, ctx, T, S, En, ref = _system(wl)
    yd = P.dense_solve(ref["ahat"], ref["bhat"])
    E = _d(En)
    rc, st = ctx.solve(E, rt.solve_opts(rt.MODE_MIXED, tol=1e-10, max_iter=20000, reduce=1))
    assert st["reduced"] == 1 and st["relres"] <= 1e-10 and st["outer_iters"] >= 1
    y = _h(E) / ref["s"]
    assert P.relres(ref["ahat"], ref["bhat"], y) <= 2e-10
    assert _full_relres(ctx, E, _d(ref["s"]), _d(ref["bhat"])) <= 2e-10
    Td, Tg = P.newton(yd * ref["s"], S, T), P.newton(_h(E), S, T)
    assert rel(Tg, Td) < 1e-6


@pytest.mark.parametrize("shape", [(67, 13, 4), (40, 9, 3)])
def test_uncolourable_grids_solve_the_full_system(shape):
    """Odd N_r (no compact halves) or odd N_phi > 1 (the periodic seam joins equal
    colours): reduce = 1 solves the full system."""
    from paper_1001_3301_amd import rt
    wl = sy.make_workload("u", *shape, 16, 10.0, clump_seed=4)
    P, ctx, T, S, En, ref = _system(wl)
    E = _d(En)
    rc, st = ctx.solve(E, rt.solve_opts(rt.MODE_FP64, tol=1e-12, reduce=1))
    assert st["reduced"] == 0 and st["relres"] <= 1e-12
    assert P.relres(ref["ahat"], ref["bhat"], _h(E) / ref["s"]) <= 1.01e-12


def test_reduced_step_against_oracle_and_deterministic():
    """Whole steps with the reduced solve: the oracle's step to 1e-13 and bitwise
    repeatability (fixed reduction order)."""
    from paper_1001_3301_amd import rt
    wl = CASES["thick-40x9x4"]()
    P = oracle.Problem.from_workload(wl)
    ctx = rt.Context.from_workload(wl)
    T0 = initial_temperature(P, wl)
    ref = P.step(wl.rho, T0, tol=1e-13, max_iter=100000)
    outs = []
    for _ in range(2):
        Td, E = _d(T0), torch.empty(P.n, dtype=torch.float64, device="cuda")
        rc, st = ctx.step(_d(wl.rho), Td, E, rt.solve_opts(rt.MODE_FP64, tol=1e-13, max_iter=100000, reduce=1))
        assert st["solve"]["reduced"] == 1
        outs.append((_h(Td), _h(E)))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert rel(outs[0][0], ref["T"]) < 1e-11
