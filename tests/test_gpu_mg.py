"""The multigrid preconditioner (rt_solve_opts.precond = 2, rt_mg_apply, rt_mg_level): an
extension of the implicit solve, not in the paper.

The hierarchy's float32 arrays (Galerkin levels, prolongation weights, phi-line
factors) are compared entry by entry with the numpy reference tests/mg_ref.py built
from the same float64 system (that reference is pinned in test_mg_ref.py), one V-cycle
with the reference's cycle, and the preconditioned solve with the oracle: its dense
Cholesky solve on small grids, its residual of the answer on a clumpy grid.
"""
import numpy as np
import pytest

import mg_ref
import oracle
from paper_1001_3301_amd import synth as sy
from _util import rel, small_workload, initial_temperature

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
    sysv = ctx.assemble(_d(wl.rho), _d(T), _d(En), _d(q))
    return P, ctx, T, S, En, ref, sysv


CASES = {
    "ragged-61x13x5-nu61": lambda: small_workload(nr=61),
    "axisym-64x16x1-nu32": lambda: sy.make_workload("a", 64, 16, 1, 32, 1.0),
    "thick-40x9x4-nu64": lambda: sy.make_workload("t", 40, 9, 4, 64, 100.0, clump_seed=3),
    "phi2-24x6x2": lambda: sy.make_workload("p2", 24, 6, 2, 16, 10.0, clump_seed=4),
    "phi3-20x7x3": lambda: sy.make_workload("p3", 20, 7, 3, 16, 10.0, clump_seed=5),
    "clumpy-64x32x64-nu16": lambda: sy.make_workload("c", 64, 32, 64, 16, 100.0, clump_seed=3000),
    "line-33x1x1": lambda: sy.make_workload("l", 33, 1, 1, 8, 1.0),
}


def _reference(ctx, sysv, shape, dtype=np.float64):
    st = ctx.system_tensors(sysv)
    return mg_ref.Hierarchy(shape, _h(st["ahat"]), _h(st["s"]), dtype=dtype)


@pytest.mark.parametrize("case", list(CASES))
def test_levels_match_the_reference(case):
    """Each level's operator, prolongation weights and line factors: the float64 set-up
    rounded to float32, against the reference's float64 values (|d| <= 1e-6 |ref| +
    1e-7 max |ref|)."""
    wl = CASES[case]()
    P, ctx, T, S, En, ref, sysv = _system(wl)
    shape = wl.grid.shape
    H = _reference(ctx, sysv, shape)
    L = len(H.levels)
    for l in range(L):
        v = ctx.mg_level(l)
        assert v["levels"] == L
        assert (v["np"], v["nt"], v["nr"]) == H.shapes[l]
        lv = H.levels[l]
        fields = {"ar": lv["ar"], "at": lv["at"], "ap": lv["ap"]}
        if l > 0:
            fields["dg"] = lv["dg"]
        else:
            assert v["dg"] is None
        if l < L - 1:
            fields["w"] = H.w[l]
            f = H.f[l]
            for k in ("im", "cp", "q", "g", "rho", "kap"):
                fields[k] = f[k]
        else:
            assert v["w"] is None and v["im"] is None
        for k, want in fields.items():
            got = _h(v[k]).astype(np.float64)
            want = np.asarray(want, dtype=np.float64).ravel()
            scale = max(np.abs(want).max(), 1e-300)
            err = np.abs(got - want) - (1e-6 * np.abs(want) + 1e-7 * scale)
            assert err.max() <= 0, (case, l, k, float(np.abs(got - want).max()), scale)


@pytest.mark.parametrize("case", list(CASES))
def test_vcycle_matches_the_reference_cycle(case):
    """rt_mg_apply (float32 inside) against the reference V-cycle in float64; the bound
    is ten times the reference's own float32-versus-float64 difference, at least 1e-5."""
    wl = CASES[case]()
    P, ctx, T, S, En, ref, sysv = _system(wl)
    shape = wl.grid.shape
    r = np.random.Generator(np.random.PCG64(23)).standard_normal(P.n)
    z = torch.empty(P.n, dtype=torch.float64, device="cuda")
    ctx.mg_apply(_d(r), z)
    torch.cuda.synchronize()
    z64 = _reference(ctx, sysv, shape).apply(r)
    z32 = _reference(ctx, sysv, shape, dtype=np.float32).apply(r)
    nrm = np.linalg.norm(z64)
    bound = max(1e-5, 10 * np.linalg.norm(z32 - z64) / nrm)
    d = np.linalg.norm(_h(z) - z64) / nrm
    print(f"{case}: |z - z_ref| / |z_ref| = {d:.2e} (reference float32: {np.linalg.norm(z32 - z64) / nrm:.2e})")
    assert d <= bound, (d, bound)


@pytest.mark.parametrize("cycle", ["K", "V", "K5"])
@pytest.mark.parametrize("case", ["ragged-61x13x5-nu61", "axisym-64x16x1-nu32", "thick-40x9x4-nu64",
                                  "phi2-24x6x2", "phi3-20x7x3", "line-33x1x1"])
def test_multigrid_solve_against_dense_oracle(case, cycle):
    """CG with one multigrid cycle per iteration (K-cycle steps on levels 1 to 3 or 1 to 5,
    or a plain V-cycle) to 1e-13 against the oracle's dense Cholesky solve of the scaled system
    (the bounds of the other float64 solves' dense tests): the oracle's residual of the
    answer, the scaled solution within 1e-8, the temperature of Eq. 16 within 1e-11."""
    from paper_1001_3301_amd import rt
    wl = CASES[case]()
    P, ctx, T, S, En, ref, sysv = _system(wl)
    E = _d(En)
    rc, st = ctx.solve(E, rt.solve_opts(rt.MODE_FP64, tol=1e-13, max_iter=2000, precond=rt.PRECOND_MG,
                                        cycle={"K": rt.CYCLE_K, "V": rt.CYCLE_V, "K5": 5}[cycle]))
    yd = P.dense_solve(ref["ahat"], ref["bhat"])
    assert st["relres"] <= 1e-13
    assert st["iters"] <= 60, st
    assert st["precond_applies"] == st["iters"]
    y = _h(E) / ref["s"]
    assert P.relres(ref["ahat"], ref["bhat"], y) <= 1.01e-13
    assert rel(y, yd) < 1e-8
    assert rel(P.newton(_h(E), S, T), P.newton(yd * ref["s"], S, T)) < 1e-11
    print(f"{case}, {cycle}-cycle: {st['iters']} iterations")
    if case == "line-33x1x1":  # the V-cycle is the exact inverse, up to its float32
        assert st["iters"] <= 2


def test_multigrid_solve_on_a_clumpy_grid_meets_the_oracle_residual():
    """64 x 32 x 64, tau550 = 100 with clumps: the oracle's own residual of the GPU's
    answer meets 1e-8, in a tenth of the iterations of float64 Jacobi CG."""
    from paper_1001_3301_amd import rt
    wl = CASES["clumpy-64x32x64-nu16"]()
    P, ctx, T, S, En, ref, sysv = _system(wl)
    E = _d(En)
    rc, st = ctx.solve(E, rt.solve_opts(rt.MODE_FP64, tol=1e-8, precond=rt.PRECOND_MG))
    E2 = _d(En)
    rc2, st2 = ctx.solve(E2, rt.solve_opts(rt.MODE_FP64, tol=1e-8))
    print(f"multigrid CG {st['iters']} iterations, Jacobi CG {st2['iters']}")
    assert st["relres"] <= 1e-8
    assert P.relres(ref["ahat"], ref["bhat"], _h(E) / ref["s"]) <= 1.05e-8
    assert 10 * st["iters"] <= st2["iters"]


@pytest.mark.parametrize("case", ["ragged-61x13x5-nu61", "axisym-64x16x1-nu32", "phi3-20x7x3", "line-33x1x1"])
def test_float32_multigrid_solve_against_dense_oracle(case):
    """Flexible CG in float32 with one V-cycle per iteration and float64 reliable updates
    (RT_SOLVE_MIXED, precond = 2) to 1e-10 (the bounds of the mixed solve's own test):
    the oracle's residual of the answer, the temperature of Eq. 16 within 1e-8 of the
    oracle's dense solve, and no more iterations than the float64 multigrid CG needs
    plus a fifth."""
    from paper_1001_3301_amd import rt
    wl = CASES[case]()
    P, ctx, T, S, En, ref, sysv = _system(wl)
    E = _d(En)
    rc, st = ctx.solve(E, rt.solve_opts(rt.MODE_MIXED, tol=1e-10, max_iter=2000, precond=rt.PRECOND_MG))
    E2 = _d(En)
    rc2, st2 = ctx.solve(E2, rt.solve_opts(rt.MODE_FP64, tol=1e-10, max_iter=2000, precond=rt.PRECOND_MG))
    yd = P.dense_solve(ref["ahat"], ref["bhat"])
    print(f"{case}: float32 FCG {st['iters']} iterations ({st['outer_iters']} reliable updates), "
          f"float64 CG {st2['iters']}")
    assert st["relres"] <= 1e-10 and st["fallback"] == 0
    assert st["precond_applies"] == st["iters"]
    assert P.relres(ref["ahat"], ref["bhat"], _h(E) / ref["s"]) <= 1.01e-10
    assert rel(P.newton(_h(E), S, T), P.newton(yd * ref["s"], S, T)) < 1e-8
    assert st["iters"] <= 1.2 * st2["iters"] + 2


def test_multigrid_rejects_other_modes():
    from paper_1001_3301_amd import rt
    wl = CASES["phi3-20x7x3"]()
    P, ctx, T, S, En, ref, sysv = _system(wl)
    for o in (rt.solve_opts(rt.MODE_GMRES, precond=2), rt.solve_opts(rt.MODE_FP64, precond=2, reduce=1),
              rt.solve_opts(rt.MODE_MIXED, precond=2, reduce=1), rt.solve_opts(rt.MODE_FP64, precond=3),
              rt.solve_opts(rt.MODE_FP64, precond=2, cycle=9), rt.solve_opts(rt.MODE_FP64, precond=2, cycle=-1)):
        rc, st = ctx.solve(_d(En), o, raise_on_error=False)
        assert rc == rt.RT_EINVAL
    with pytest.raises(Exception):
        ctx.mg_level(99)
