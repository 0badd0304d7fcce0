"""Seeded synthetic inputs for the radiation step (grid, star, opacities, density).

This module builds the *inputs* of the method and nothing else: it holds none of
the method's arithmetic (no ray trace, no diffusion operator, no solve).  Both the
HIP path and the CPU oracle consume what it returns, so it is kept free of either.

What it stands in for (Sect. "Physical setup of the star, the disk, and the
envelope" and "Numerical setup" of Kuiper et al.):

* star: T_* = 5800 K, R_* = 1 R_sun;
* spherical-polar grid, radially log-stretched from 1 AU to 1000 AU, polar-uniform
  over [0, pi], azimuthally uniform over [0, 2 pi);
* flared disk rho0 (r_d/R) exp(-(pi/4)(z/h)^2), h = z_d (R/r_d)^1.125 with
  r_d = 500 AU, z_d = 125 AU (the six density-setup equations), evaluated with the
  cylindrical R = r sin(theta), z = r cos(theta) at cell centres, plus a spherical
  envelope 1e-3 rho0 (r/r_d)^-1.5, floored at 1e-100 of the maximum density;
* rho0 chosen so the midplane optical depth at 550 nm equals tau550 (the rho0 table
  of that section); the published Draine & Lee opacities are replaced by a power law
  kappa_nu = kappa0 (nu/nu550)^beta with a plateau above 1e15 Hz, tabulated on 64
  temperatures with a sublimation drop at 1500 K; its Planck and Rosseland means are
  tabulated too, as the paper tabulates them for its dust model;
* lognormal clumps (sigma_ln rho = 0.5, Gaussian correlation of 8 cells).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# CGS constants (CODATA 2018 exact/recommended values).
C_LIGHT = 2.99792458e10
H_PLANCK = 6.62607015e-27
K_BOLTZ = 1.380649e-16
SIGMA_SB = 5.670374419e-5
A_RAD = 4.0 * SIGMA_SB / C_LIGHT
AU = 1.495978707e13
R_SUN = 6.957e10
M_SUN = 1.98841e33
M_H = 1.6735575e-24

T_STAR = 5800.0
R_STAR = R_SUN
R_MIN = 1.0 * AU
R_MAX = 1000.0 * AU
R_D = 500.0 * AU
Z_D = 125.0 * AU
NU_550 = C_LIGHT / 550e-7
KAPPA0 = 232.59          # cm^2/g at 550 nm; reproduces the paper's rho0 <-> tau550 table
BETA = 1.5
NU_PLATEAU = 1e15
T_SUBLIMATION = 1500.0
SUBLIMATION_FACTOR = 1e-8
T_BC = 14.7              # outer Dirichlet temperature
C_V = 1.5 * K_BOLTZ / (2.33 * M_H)   # erg g^-1 K^-1 for a mean molecular weight of 2.33
DT_DEFAULT = 1e9


@dataclass
class Grid:
    """Cell faces of the spherical-polar grid (host arrays, float64)."""
    r_face: np.ndarray
    th_face: np.ndarray
    ph_face: np.ndarray

    @property
    def shape(self):
        return (len(self.r_face) - 1, len(self.th_face) - 1, len(self.ph_face) - 1)

    @property
    def ncell(self):
        nr, nt, npp = self.shape
        return nr * nt * npp

    def centres(self):
        rf, tf, pf = self.r_face, self.th_face, self.ph_face
        return 0.5 * (rf[1:] + rf[:-1]), 0.5 * (tf[1:] + tf[:-1]), 0.5 * (pf[1:] + pf[:-1])


@dataclass
class Opacity:
    """Opacity table: kappa[n_T, n_nu] at mid-frequencies nu, plus Planck/Rosseland means."""
    T: np.ndarray
    nu: np.ndarray
    kappa: np.ndarray
    kappa_P: np.ndarray
    kappa_R: np.ndarray


@dataclass
class Workload:
    name: str
    grid: Grid
    opacity: Opacity
    R_star: float
    T_star: float
    rho: np.ndarray             # (n_ph, n_th, n_r) float64, r fastest
    tau550: float
    rho0: float
    dt: float = DT_DEFAULT
    c_V: float = C_V
    T_bc: float = T_BC
    E_floor: float = A_RAD * 1.0
    meta: dict = field(default_factory=dict)


def make_grid(nr: int, nt: int, nph: int, r_min: float = R_MIN, r_max: float = R_MAX) -> Grid:
    """Log-spaced radial faces, uniform polar faces on [0, pi], uniform azimuth on [0, 2 pi)."""
    rf = np.geomspace(r_min, r_max, nr + 1)
    rf[0], rf[-1] = r_min, r_max
    tf = np.pi * np.arange(nt + 1) / nt
    pf = 2.0 * np.pi * np.arange(nph + 1) / nph
    return Grid(rf, tf, pf)


def frequencies(n_nu: int, lo: float = 1e11, hi: float = 3e15) -> np.ndarray:
    """Log-spaced bin mid-frequencies."""
    return np.geomspace(lo, hi, n_nu)


def _kappa_nu_cont(nu, kappa0=KAPPA0, beta=BETA, nu_p=NU_PLATEAU):
    return kappa0 * (np.minimum(nu, nu_p) / NU_550) ** beta


def _mean_opacities_cont(T, kappa0=KAPPA0, beta=BETA, nu_p=NU_PLATEAU):
    """Planck and Rosseland means of the continuous power law by quadrature in x = h nu/kT."""
    from scipy import integrate

    xp = H_PLANCK * nu_p / (K_BOLTZ * T)
    scale = kappa0 * (K_BOLTZ * T / (H_PLANCK * NU_550)) ** beta   # kappa at x = 1
    kap_plat = kappa0 * (nu_p / NU_550) ** beta

    def kap(x):
        return scale * x ** beta if x < xp else kap_plat

    def planck(x):
        if x <= 0:
            return 0.0
        if x > 700:
            return x ** 3 * math.exp(-x)
        return x ** 3 / math.expm1(x)

    def dbdt(x):
        if x <= 0:
            return 0.0
        if x > 1.0:
            e = math.exp(-x)
            return x ** 4 * e / ((1.0 - e) * (1.0 - e))
        em = math.expm1(x)
        return x ** 4 * (em + 1.0) / (em * em)

    pts = [p for p in (xp,) if 0 < p < 800]
    quad = dict(limit=400, epsabs=0.0, epsrel=1e-13)
    num = integrate.quad(lambda x: kap(x) * planck(x), 0, 800, points=pts or None, **quad)[0]
    den = math.pi ** 4 / 15.0
    kP = num / den
    inv = integrate.quad(lambda x: dbdt(x) / kap(x) if x > 0 else 0.0, 0, 800,
                         points=pts or None, **quad)[0]
    den_r = 4.0 * math.pi ** 4 / 15.0
    kR = den_r / inv
    return kP, kR


def make_opacity(nu: np.ndarray, n_T: int = 64, T_lo: float = 1.0, T_hi: float = 1e4,
                 kappa0: float = KAPPA0, beta: float = BETA, nu_p: float = NU_PLATEAU,
                 T_sub: float = T_SUBLIMATION, eps: float = SUBLIMATION_FACTOR) -> Opacity:
    """Synthetic dust opacity table (stand-in for Draine & Lee 1984).

    kappa_nu(T_k) = eps_k * kappa0 * (min(nu, nu_p)/nu550)^beta, with eps_k = 1 below the
    sublimation temperature and `eps` at or above it; Planck/Rosseland means by quadrature
    of the continuous spectrum (not of the bins), times the same eps_k.
    """
    T = np.geomspace(T_lo, T_hi, n_T)
    eps_k = np.where(T < T_sub, 1.0, eps)
    kap_nu = _kappa_nu_cont(np.asarray(nu, dtype=np.float64), kappa0, beta, nu_p)
    kappa = eps_k[:, None] * kap_nu[None, :]
    kP = np.empty(n_T)
    kR = np.empty(n_T)
    for k, t in enumerate(T):
        p, r = _mean_opacities_cont(t, kappa0, beta, nu_p)
        kP[k] = eps_k[k] * p
        kR[k] = eps_k[k] * r
    return Opacity(T, np.asarray(nu, dtype=np.float64).copy(), np.ascontiguousarray(kappa), kP, kR)


def rho0_for_tau(tau550: float, kappa550: float = KAPPA0, envelope: float = 1e-3,
                 r_min: float = R_MIN, r_max: float = R_MAX, r_d: float = R_D) -> float:
    """rho0 such that the analytic midplane optical depth at 550 nm (disk + envelope) is tau550."""
    disk = r_d * math.log(r_max / r_min)
    env = envelope * 2.0 * r_d * ((r_min / r_d) ** -0.5 - (r_max / r_d) ** -0.5)
    return tau550 / (kappa550 * (disk + env))


def density_smooth(grid: Grid, rho0: float, envelope: float = 1e-3, floor_rel: float = 1e-100) -> np.ndarray:
    """Disk + envelope density at cell centres, shape (n_ph, n_th, n_r) (r fastest)."""
    rc, tc, _ = grid.centres()
    nr, nt, nph = grid.shape
    r = rc[None, :]
    th = tc[:, None]
    R = r * np.sin(th)
    z = r * np.cos(th)
    h = Z_D * (R / R_D) ** 1.125
    with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
        disk = rho0 * (R_D / R) * np.exp(-(np.pi / 4.0) * (z / h) ** 2)
    disk = np.nan_to_num(disk, nan=0.0, posinf=0.0)
    env = envelope * rho0 * (r / R_D) ** -1.5 * np.ones_like(th)
    rho2 = disk + env
    rho2 = np.maximum(rho2, floor_rel * rho2.max())
    return np.ascontiguousarray(np.broadcast_to(rho2[None, :, :], (nph, nt, nr)))


def clump_field(shape, seed: int, corr: float = 8.0) -> np.ndarray:
    """Zero-mean, unit-variance Gaussian random field with covariance exp(-d^2/(2 corr^2)).

    White noise from PCG64(seed), filtered in Fourier space (periodic, index units) by the
    square root of the covariance spectrum, then normalised to sample mean 0 / variance 1.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal(shape)
    spec = np.fft.rfftn(g)
    kk = None
    for ax, n in enumerate(shape):
        if ax == len(shape) - 1:
            k = 2.0 * np.pi * np.fft.rfftfreq(n)
        else:
            k = 2.0 * np.pi * np.fft.fftfreq(n)
        sh = [1] * len(shape)
        sh[ax] = len(k)
        k2 = (k ** 2).reshape(sh)
        kk = k2 if kk is None else kk + k2
    spec *= np.exp(-0.25 * kk * corr * corr)
    g = np.fft.irfftn(spec, s=shape, axes=tuple(range(len(shape))))
    g -= g.mean()
    sd = g.std()
    if sd > 0:
        g /= sd
    return g


def apply_clumps(rho: np.ndarray, seed: int, sigma: float = 0.5, corr: float = 8.0) -> np.ndarray:
    """Lognormal clumps: rho * exp(sigma g - sigma^2/2) with g from clump_field."""
    g = clump_field(rho.shape, seed, corr)
    return np.ascontiguousarray(rho * np.exp(sigma * g - 0.5 * sigma * sigma))


def make_workload(name: str, nr: int, nt: int, nph: int, n_nu: int, tau550: float,
                  clump_seed: int | None = None, dt: float = DT_DEFAULT) -> Workload:
    grid = make_grid(nr, nt, nph)
    nu = frequencies(n_nu)
    op = make_opacity(nu)
    rho0 = rho0_for_tau(tau550)
    rho = density_smooth(grid, rho0)
    if clump_seed is not None:
        rho = apply_clumps(rho, clump_seed)
    return Workload(name, grid, op, R_STAR, T_STAR, rho, tau550, rho0, dt=dt,
                    meta=dict(clump_seed=clump_seed, n_nu=n_nu))


# The named workloads.  Sizes are (N_r, N_theta, N_phi), N_nu.
CONFIGS = {
    "axisym-64x16x1-nu32": dict(nr=64, nt=16, nph=1, n_nu=32, taus=(1.0,), seeds=(None,)),
    "clumpy-128x64x128-nu64": dict(nr=128, nt=64, nph=128, n_nu=64, taus=(0.1, 1.0, 10.0, 100.0),
                                    seeds=(1000, 1001, 1002, 1003)),
    "clumpy-256x128x256-nu64": dict(nr=256, nt=128, nph=256, n_nu=64, taus=(100.0,), seeds=(3000,)),
    "clumpy-512x256x512-nu64": dict(nr=512, nt=256, nph=512, n_nu=64, taus=(100.0,), seeds=(5000,)),
    # one GPU's share of the 512x256x512 grid split into eight phi-slabs, at its shape
    # (generated as a whole periodic grid, so kernel times carry over, iteration counts
    # do not)
    "clumpy-512x256x64-nu64": dict(nr=512, nt=256, nph=64, n_nu=64, taus=(100.0,), seeds=(5001,)),
}


def config_workloads(name: str):
    c = CONFIGS[name]
    return [make_workload(name, c["nr"], c["nt"], c["nph"], c["n_nu"], t, s)
            for t, s in zip(c["taus"], c["seeds"])]
