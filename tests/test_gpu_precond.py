"""The radial-line block-Jacobi comparator (rt_solve_opts.precond = 1): the block-Jacobi
class of preconditioner of the paper's solver set-up, with each radial row's tridiagonal
block solved exactly.

The preconditioner application is checked by a property of the exact block solve (the
oracle's assembled radial couplings applied to z give back r), the preconditioned solve
against the oracle's dense Cholesky solve of the full system.
"""
import numpy as np
import pytest

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
    ctx.assemble(_d(wl.rho), _d(T), _d(En), _d(q))
    return P, ctx, T, S, En, ref


CASES = {
    "ragged-61x13x5-nu61": lambda: small_workload(nr=61),
    "axisym-64x16x1-nu32": lambda: sy.make_workload("a", 64, 16, 1, 32, 1.0),
    "thick-40x9x4-nu64": lambda: sy.make_workload("t", 40, 9, 4, 64, 100.0, clump_seed=3),
}


@pytest.mark.parametrize("case", list(CASES))
def test_line_block_solve_inverts_the_radial_blocks(case):
    wl = CASES[case]()
    P, ctx, T, S, En, ref = _system(wl)
    nr, nt, npp = wl.grid.shape
    r = np.random.Generator(np.random.PCG64(17)).standard_normal(P.n)
    z = torch.empty(P.n, dtype=torch.float64, device="cuda")
    ctx.precond_apply(_d(r), z)
    torch.cuda.synchronize()
    zz = _h(z).reshape(npp, nt, nr)
    a = ref["ahat"].reshape(3, npp, nt, nr)[0]
    Tz = zz.copy()
    Tz[..., :-1] += a[..., :-1] * zz[..., 1:]
    Tz[..., 1:] += a[..., :-1] * zz[..., :-1]
    assert np.max(np.abs(Tz.ravel() - r)) <= 1e-12 * np.max(np.abs(r))


@pytest.mark.parametrize("case", list(CASES))
def test_line_preconditioned_solve_against_dense_oracle(case):
    from paper_1001_3301_amd import rt
    wl = CASES[case]()
    P, ctx, T, S, En, ref = _system(wl)
    yd = P.dense_solve(ref["ahat"], ref["bhat"])
    E = _d(En)
    rc, st = ctx.solve(E, rt.solve_opts(rt.MODE_FP64, tol=1e-13, max_iter=20000, check_every=8, precond=1))
    assert st["relres"] <= 1e-13
    y = _h(E) / ref["s"]
    assert P.relres(ref["ahat"], ref["bhat"], y) <= 1.01e-13
    assert rel(y, yd) < 1e-8
    assert rel(P.newton(_h(E), S, T), P.newton(yd * ref["s"], S, T)) < 1e-11
    E2 = _d(En)
    rc, s2 = ctx.solve(E2, rt.solve_opts(rt.MODE_FP64, tol=1e-13, max_iter=20000, check_every=8))
    print(f"{case}: line block Jacobi {st['iters']} iterations, Jacobi {s2['iters']}")
    assert st["iters"] <= s2["iters"]


def test_line_preconditioner_rejects_other_modes():
    from paper_1001_3301_amd import rt
    wl = CASES["thick-40x9x4-nu64"]()
    P, ctx, T, S, En, ref = _system(wl)
    for o in (rt.solve_opts(rt.MODE_MIXED, precond=1), rt.solve_opts(rt.MODE_FP64, precond=1, reduce=1),
              rt.solve_opts(rt.MODE_FP64, precond=3)):
        rc, _ = ctx.solve(_d(En), o, raise_on_error=False)
        assert rc == rt.RT_EINVAL
