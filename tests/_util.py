"""Shared helpers of the parity tests."""
import numpy as np

from paper_1001_3301_amd import synth as sy


def rel(x, y):
    """max_i |x_i - y_i| / max(|y_i|, 1e-30 max|y|)."""
    x = np.asarray(x, dtype=np.float64).ravel()
    y = np.asarray(y, dtype=np.float64).ravel()
    floor = 1e-30 * max(np.max(np.abs(y)), 1e-300)
    return float(np.max(np.abs(x - y) / np.maximum(np.abs(y), floor)))


def small_workload(nr=67, nt=13, nph=5, n_nu=61, tau=10.0, seed=21, dt=1e9):
    """A ragged grid (sizes prime to every tile) with clumps."""
    return sy.make_workload(f"ragged-{nr}x{nt}x{nph}-nu{n_nu}", nr, nt, nph, n_nu, tau,
                            clump_seed=seed, dt=dt)


def initial_temperature(P, wl):
    """T^0 of the oracle: Newton on Eq. 16 with E = a T_bc^4 and the irradiation at T_bc."""
    T0 = np.full(P.n, wl.T_bc)
    q, S, _ = P.raytrace(wl.rho, T0, want_faces=False)
    E0 = np.full(P.n, sy.A_RAD * wl.T_bc ** 4)
    return P.newton(E0, S, T0)


def seeded_temperature(n, seed, lo=15.0, hi=700.0):
    """Seeded temperature field for kernel-level parity (not a method result)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.exp(rng.uniform(np.log(lo), np.log(hi), n))
