"""The 256 x 128 x 256-cell, 64-bin workload (tau550 = 100, clumps seed 3000) against
the oracle, whole grid: one radiation step from the prepared state (irradiation at
T_bc, then Eq. 16 with E = a T_bc^4) by the plain float64 solve, the reduced
mixed-precision solve and the learned solve with the reduced mixed finish, each to the
relative residual 1e-8, against the oracle's step solved to 1e-10 (the OpenMP build of
the oracle, which sums its dot products in fixed blocks).

For every mode: the oracle's own assembly and residual of the GPU's E (<= tol), and the
errors of T, E_R and the radiative force against the oracle's step, printed and bounded:
T within 1e-3 (the reduced-precision bar; the float64 mode within 1e-6), E_R within
cond(A^) x tol of the oracle's E.  The prepared state itself (ray trace, Newton) is
compared cell by cell over the whole grid.
"""
import numpy as np
import pytest

import oracle
from paper_1001_3301_amd import synth as sy

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

A = sy.A_RAD
CONFIG = "clumpy-256x128x256-nu64"


def _maxrel(got, ref):
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)))


@pytest.fixture(scope="module")
def c3():
    from paper_1001_3301_amd import rt
    wl = sy.config_workloads(CONFIG)[0]
    print(f"\n{CONFIG}: oracle with {oracle.threads()} threads", flush=True)
    P = oracle.Problem.from_workload(wl, parallel=True)
    rho = wl.rho.ravel()
    T0 = np.full(P.n, wl.T_bc)
    _, S, _ = P.raytrace(rho, T0, want_faces=False)
    T0 = P.newton(np.full(P.n, A * wl.T_bc ** 4), S, T0)
    q, S, _ = P.raytrace(rho, T0, want_faces=False)
    En = P.energy(T0, S)
    sysref = P.assemble(rho, T0, En, q)
    ref = P.step(rho, T0, tol=1e-10)
    assert ref["status"] == 0
    print(f"oracle step: {ref['iters']} CG iterations to {ref['relres']:.2e}", flush=True)
    ctx = rt.Context.from_workload(wl)
    n = ctx.n
    rho_d = torch.tensor(rho, device="cuda")
    T0_d = torch.full((n,), wl.T_bc, dtype=torch.float64, device="cuda")
    q_d = torch.empty(n, dtype=torch.float64, device="cuda")
    S_d = torch.empty_like(q_d)
    ctx.raytrace(rho_d, T0_d, q_d, S_d)
    ctx.temperature(torch.full((n,), A * wl.T_bc ** 4, dtype=torch.float64, device="cuda"), S_d, T0_d)
    torch.cuda.synchronize()
    return wl, P, ctx, rho_d, T0_d, dict(T0=T0, S=S, q=q, En=En, sys=sysref, ref=ref)


def test_c3_prepared_state_whole_grid(c3):
    """Ray trace at T_bc and the Newton temperature of the prepared state, every cell."""
    wl, P, ctx, rho_d, T0_d, O = c3
    assert _maxrel(T0_d.cpu().numpy(), O["T0"]) < 1e-11


def _small_trained_net():
    from paper_1001_3301_amd import rt
    wl = sy.make_workload("train-64x32x32", 64, 32, 32, 64, 100.0, clump_seed=3001)
    ctx = rt.Context.from_workload(wl)
    n = ctx.n
    rho = torch.tensor(wl.rho.ravel(), device="cuda")
    T = torch.full((n,), wl.T_bc, dtype=torch.float64, device="cuda")
    q = torch.empty(n, dtype=torch.float64, device="cuda")
    S = torch.empty_like(q)
    ctx.raytrace(rho, T, q, S)
    ctx.temperature(torch.full((n,), A * wl.T_bc ** 4, dtype=torch.float64, device="cuda"), S, T)
    ctx.raytrace(rho, T, q, S)
    En = torch.empty_like(q)
    ctx.energy(T, S, En)
    ctx.assemble(rho, T, En, q)
    ds = rt.Dataset(ctx, 4)
    ds.add(En, [0, 10, 40, 150])
    net = rt.Net(seed=3)
    net.train(ctx, ds, epochs=8, lr=1e-3, seed=1, loss=rt.LOSS_RESIDUAL)
    return net, ds, ctx


@pytest.mark.parametrize("mode", ["fp64", "mixed-rb", "learned-rb"])
def test_c3_step_against_oracle(c3, mode):
    from paper_1001_3301_amd import rt
    wl, P, ctx, rho_d, T0_d, O = c3
    n = ctx.n
    keep = None
    if mode == "fp64":
        opts = rt.solve_opts(rt.MODE_FP64, tol=1e-8)
    elif mode == "mixed-rb":
        opts = rt.solve_opts(rt.MODE_MIXED, tol=1e-8, reduce=1)
    else:
        keep = _small_trained_net()
        opts = rt.solve_opts(rt.MODE_LEARNED, tol=1e-8, net=keep[0], inner_max_iter=5, reduce=1)
    T = T0_d.clone()
    E = torch.empty(n, dtype=torch.float64, device="cuda")
    f = torch.empty(4 * n, dtype=torch.float64, device="cuda")
    rc, st = ctx.step(rho_d, T, E, opts, f_rad=f)
    torch.cuda.synchronize()
    sv = st["solve"]
    assert rc == rt.RT_OK and sv["fallback"] == 0
    ref, sysref = O["ref"], O["sys"]
    Eg, Tg, fg = E.cpu().numpy(), T.cpu().numpy(), f.cpu().numpy().reshape(4, n)
    fr = ref["force"].reshape(4, n)
    res = P.relres(sysref["ahat"], sysref["bhat"], Eg / sysref["s"])
    eT = _maxrel(Tg, ref["T"])
    eE = _maxrel(Eg, ref["E"])
    eE2 = float(np.linalg.norm(Eg - ref["E"]) / np.linalg.norm(ref["E"]))
    ef = [float(np.max(np.abs(fg[c] - fr[c])) / np.max(np.abs(fr[c]))) for c in range(4)]
    print(f"{mode}: {sv['iters']} iterations ({sv['precond_applies']} network applications), "
          f"oracle relres {res:.3e}; vs the oracle step at 1e-10: T {eT:.2e}, E_R max {eE:.2e} "
          f"(L2 {eE2:.2e}), force r/theta/phi {ef[1]:.2e}/{ef[2]:.2e}/{ef[3]:.2e} of max, stellar {ef[0]:.2e}")
    assert res <= 1.05e-8
    assert eT <= (1e-6 if mode == "fp64" else 1e-3)
    assert eE2 <= 1e-4
    assert ef[0] <= 1e-10
    assert max(ef[1:]) <= 1e-4
