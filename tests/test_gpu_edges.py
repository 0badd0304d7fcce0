"""Degenerate grids against the oracle: the fewest radial cells the library accepts
(N_r = 2, one black and one red cell per radial row), a single polar row, a single
column, N_phi = 2 (both phi faces of a cell join the same neighbour), few bins, and
columns near the longest the library accepts.

Every kernel of the step runs at these sizes with most of its threads idle or clamped:
the ray trace (one partial segment per column), the assembly's boundary faces, the
Krylov kernels with every neighbour a boundary (full system from graphs, the reduced
system in one workgroup and from graphs in float32, GMRES(30) whose Krylov space fills
up within one cycle, the multigrid CG with hierarchies of one to three levels), Newton
and the force.
"""
import numpy as np
import pytest

import oracle
from paper_1001_3301_amd import synth as sy
from _util import rel, initial_temperature

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# ... and long columns: 1472 cells for whole steps (the oracle's dense solve), the
# longest the ray trace's LDS takes (N_r <= 2944) for the ray trace
SHAPES = [(2, 1, 1), (2, 3, 1), (4, 2, 2), (6, 1, 4), (10, 7, 2), (1472, 2, 1)]
RT_SHAPES = SHAPES + [(2944, 2, 1)]


def _d(x):
    return torch.tensor(np.ascontiguousarray(x, dtype=np.float64).ravel(), device="cuda")


def _h(t):
    return t.detach().cpu().numpy()


def _wl(shape):
    return sy.make_workload("edge", *shape, 4, 10.0, clump_seed=31)


@pytest.mark.parametrize("shape", RT_SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_tiny_raytrace_parity(shape):
    from paper_1001_3301_amd import rt
    wl = _wl(shape)
    P = oracle.Problem.from_workload(wl)
    ctx = rt.Context.from_workload(wl)
    T = initial_temperature(P, wl) * np.linspace(0.9, 3.0, P.n)
    q0, S0, F0, Fnu0 = P.raytrace(wl.rho, T, want_bins=True)
    nr, nt, npp = shape
    q, S = (torch.empty(P.n, dtype=torch.float64, device="cuda") for _ in range(2))
    Ff = torch.empty((nr + 1) * nt * npp, dtype=torch.float64, device="cuda")
    Fnu = torch.empty((nr + 1) * nt * npp * 4, dtype=torch.float64, device="cuda")
    ctx.raytrace(_d(wl.rho), _d(T), q, S, Ff, Fnu)
    torch.cuda.synchronize()
    assert rel(_h(q), q0) < 1e-11
    assert rel(_h(S), S0) < 1e-11
    assert rel(_h(Ff), F0) < 1e-11
    assert rel(_h(Fnu), Fnu0) < 1e-11


def test_column_length_limit():
    """rt_create takes columns up to the ray trace's LDS limit and refuses longer ones."""
    from paper_1001_3301_amd import rt
    th, ph = np.array([0.4, 0.5]), np.array([0.0, 0.1])
    rt.Context(np.linspace(1.0, 2.0, 2945), th, ph, 64).close()
    with pytest.raises(rt.RtError) as ei:
        rt.Context(np.linspace(1.0, 2.0, 2946), th, ph, 64)
    assert ei.value.status == rt.RT_EINVAL and "2944" in str(ei.value)


MODES = {  # name: (mode, reduce, solve tol, T bar[, further solve options])
    "fp64": (0, 0, 1e-12, 1e-11),
    "fp64-rb": (0, 1, 1e-12, 1e-11),
    "mixed-rb": (1, 1, 1e-12, 1e-9),
    # GMRES(30): on the smallest grids the Krylov space fills up within a cycle; solved
    # to 1e-13, since its 1e-12 residual leaves T 1.6e-11 off on the 1472-cell columns
    "gmres": (3, 0, 1e-13, 1e-11),
    # the multigrid CG: hierarchies of one to three levels, lines of one, two and four
    # phi cells, single theta rows, the coarsest line of 1472 cells
    "fp64-mg": (0, 0, 1e-12, 1e-11, dict(precond=2)),
    "fp64-mgv": (0, 0, 1e-12, 1e-11, dict(precond=2, cycle=1)),
    "mixed-mg": (1, 0, 1e-12, 1e-9, dict(precond=2)),
}


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_tiny_step_parity(shape, mode):
    from paper_1001_3301_amd import rt
    m, rb, tol, bar = MODES[mode][:4]
    extra = MODES[mode][4] if len(MODES[mode]) > 4 else {}
    wl = _wl(shape)
    P = oracle.Problem.from_workload(wl)
    ctx = rt.Context.from_workload(wl)
    T0 = initial_temperature(P, wl)
    ref = P.step(wl.rho, T0, dense=True)  # the oracle's exact (Cholesky) solve: n <= 2944 here
    Td = _d(T0)
    E = torch.empty(P.n, dtype=torch.float64, device="cuda")
    f = torch.empty(4 * P.n, dtype=torch.float64, device="cuda")
    rc, st = ctx.step(_d(wl.rho), Td, E, rt.solve_opts(m, tol=tol, max_iter=100000, reduce=rb, **extra), f_rad=f)
    assert rc == 0 and st["solve"]["relres"] <= tol
    assert st["solve"]["reduced"] == rb
    assert rel(_h(Td), ref["T"]) < bar
    fr, fg = ref["force"].reshape(4, P.n), _h(f).reshape(4, P.n)
    assert rel(fg[0], fr[0]) < 1e-11
