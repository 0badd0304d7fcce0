"""ctypes front end of the serial FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU-baseline
leg of the benchmark, never by the product package.  All arrays are host numpy
float64 arrays in the r-fastest layout c = i + N_r (j + N_theta k).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SRC_NN = os.path.join(_HERE, "oracle_nn.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (serial, -O2, no FMA contraction) and the
    same sources with OpenMP into liboracle_omp.so (the all-cores CPU baseline and the
    oracle side of the tests on the largest grids)."""
    for path, extra in ((_LIB, ["-Wno-unknown-pragmas"]), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                                   "-std=c99", "-Wall", *extra, "-o", tmp, _SRC, _SRC_NN, "-lm"])
            os.replace(tmp, path)
    return _LIB


class _Grid(C.Structure):
    _fields_ = [("nr", C.c_int), ("nt", C.c_int), ("np", C.c_int),
                ("rf", C.POINTER(C.c_double)), ("tf", C.POINTER(C.c_double)),
                ("pf", C.POINTER(C.c_double))]


class _Opac(C.Structure):
    _fields_ = [("nT", C.c_int), ("nnu", C.c_int), ("T", C.POINTER(C.c_double)),
                ("kap", C.POINTER(C.c_double)), ("kapP", C.POINTER(C.c_double)),
                ("kapR", C.POINTER(C.c_double))]


class _Star(C.Structure):
    _fields_ = [("R", C.c_double), ("Teff", C.c_double), ("F0", C.POINTER(C.c_double))]


class _Fld(C.Structure):
    _fields_ = [("dt", C.c_double), ("cV", C.c_double), ("Tbc", C.c_double),
                ("Efloor", C.c_double)]


_libs = {}


def lib(parallel: bool = False):
    """The serial oracle library, or (parallel=True) its OpenMP build."""
    if parallel not in _libs:
        path = _LIB_OMP if parallel else _LIB
        if not os.path.exists(path) or os.path.getmtime(path) < max(os.path.getmtime(_SRC),
                                                                   os.path.getmtime(_SRC_NN)):
            build()
        L = C.CDLL(path)
        P = C.POINTER
        dp = P(C.c_double)
        L.og_star_bins.argtypes = [C.c_double, C.c_int, dp, dp]
        L.og_raytrace.argtypes = [P(_Grid), P(_Opac), P(_Star), dp, dp, dp, dp, dp, dp]
        L.og_energy.argtypes = [P(_Grid), P(_Opac), P(_Fld), dp, dp, dp]
        L.og_assemble.argtypes = [P(_Grid), P(_Opac), P(_Fld), dp, dp, dp, dp, dp,
                                  dp, dp, dp, dp, dp, dp]
        L.og_relax.argtypes = [P(_Grid), P(_Opac), P(_Star), P(_Fld), dp, dp, dp, C.c_int, C.c_double, C.c_int,
                               C.c_int, C.c_double, dp]
        L.og_gray_table.argtypes = [P(_Opac), dp, dp]
        L.og_tau_rosseland.argtypes = [P(_Grid), P(_Opac), dp, dp, dp]
        L.og_gray_table.restype = C.c_double
        L.og_gmres.argtypes = [P(_Grid), dp, dp, dp, C.c_int, C.c_double, C.c_int, P(C.c_int), P(C.c_double)]
        L.og_spmv.argtypes = [P(_Grid), dp, dp, dp]
        L.og_relres.argtypes = [P(_Grid), dp, dp, dp]
        L.og_relres.restype = C.c_double
        L.og_cg.argtypes = [P(_Grid), dp, dp, dp, C.c_double, C.c_int, P(C.c_int), dp]
        L.og_dense_solve.argtypes = [P(_Grid), dp, dp, dp]
        L.og_newton.argtypes = [P(_Grid), P(_Opac), dp, dp, dp]
        L.og_force.argtypes = [P(_Grid), P(_Opac), P(_Fld), dp, dp, dp, dp, dp, dp]
        L.og_step.argtypes = [P(_Grid), P(_Opac), P(_Star), P(_Fld), dp, dp, dp, dp,
                              C.c_double, C.c_int, C.c_int, P(C.c_int), dp]
        L.og_kappa_nu.argtypes = [P(_Opac), C.c_double, C.c_int]
        L.og_kappa_nu.restype = C.c_double
        L.og_kappa_P.argtypes = [P(_Opac), C.c_double]
        L.og_kappa_P.restype = C.c_double
        L.og_kappa_R.argtypes = [P(_Opac), C.c_double]
        L.og_kappa_R.restype = C.c_double
        L.og_const_a.restype = C.c_double
        ip = C.c_int
        L.ognn_conv_fwd.argtypes = [ip, ip, ip, dp, ip, dp, dp, ip, ip, dp]
        L.ognn_conv_bwd_data.argtypes = [ip, ip, ip, dp, ip, dp, ip, dp]
        L.ognn_conv_bwd_weight.argtypes = [ip, ip, ip, dp, ip, dp, ip, dp, dp]
        L.ognn_pool.argtypes = [ip, ip, ip, dp, ip, dp]
        L.ognn_up.argtypes = [ip, ip, ip, dp, ip, dp]
        L.ognn_param_offset.argtypes = [ip]
        L.ognn_param_offset.restype = C.c_long
        L.ognn_param_count.restype = C.c_long
        for f in ("ognn_cin", "ognn_cout", "ognn_taps"):
            getattr(L, f).argtypes = [ip]
        L.ognn_forward_bf16.argtypes = [ip, ip, ip, dp, dp, dp]
        L.ognn_bf16_round.argtypes = [C.c_double]
        L.ognn_bf16_round.restype = C.c_double
        L.ognn_loss_grad.argtypes = [ip, ip, ip, dp, dp, dp, dp, dp]
        L.ognn_loss_grad.restype = C.c_double
        L.ognn_loss_grad_resid.argtypes = [ip, ip, ip, dp, dp, dp, dp, dp, dp]
        L.ognn_loss_grad_resid.restype = C.c_double
        L.ognn_loss.argtypes = [C.c_long, dp, dp, dp]
        L.ognn_loss.restype = C.c_double
        L.ognn_adam.argtypes = [C.c_long, dp, dp, dp, dp, C.c_double, C.c_double, C.c_double,
                                C.c_double, ip]
        L.og_const_c.restype = C.c_double
        L.og_threads.restype = C.c_int
        _libs[parallel] = L
    return _libs[parallel]


def threads(parallel: bool = True) -> int:
    """Threads the (parallel) oracle's loops use."""
    return lib(parallel).og_threads()


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _p(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


class Problem:
    """Holds the ctypes views of grid / opacity / star / FLD parameters for one problem."""

    def __init__(self, r_face, th_face, ph_face, T_tab, kappa, kappa_P, kappa_R,
                 R_star=None, F0=None, T_star=None, dt=1e9, c_V=None, T_bc=14.7, E_floor=None,
                 parallel=False):
        self.L = lib(parallel)
        self._keep = [_f64(x) for x in (r_face, th_face, ph_face, T_tab, kappa, kappa_P, kappa_R)]
        rf, tf, pf, Tt, kap, kP, kR = self._keep
        self.shape = (len(rf) - 1, len(tf) - 1, len(pf) - 1)
        self.n = int(np.prod(self.shape))
        self.g = _Grid(self.shape[0], self.shape[1], self.shape[2], _p(rf), _p(tf), _p(pf))
        self.op = _Opac(len(Tt), kap.shape[1], _p(Tt), _p(kap), _p(kP), _p(kR))
        self.nnu = kap.shape[1]
        a = self.L.og_const_a()
        self.F0 = None if F0 is None else _f64(F0)
        self.st = _Star(R_star or 0.0, T_star or 0.0, _p(self.F0))
        self.fld = _Fld(dt, c_V if c_V is not None else 0.0, T_bc,
                        E_floor if E_floor is not None else a * 1.0)

    @classmethod
    def from_workload(cls, wl, F0=None, parallel=False):
        if F0 is None:
            F0 = star_bins(wl.T_star, wl.opacity.nu)
        g, op = wl.grid, wl.opacity
        return cls(g.r_face, g.th_face, g.ph_face, op.T, op.kappa, op.kappa_P, op.kappa_R,
                   R_star=wl.R_star, F0=F0, T_star=wl.T_star, dt=wl.dt, c_V=wl.c_V,
                   T_bc=wl.T_bc, E_floor=wl.E_floor, parallel=parallel)

    # --- per-step pieces -------------------------------------------------
    def raytrace(self, rho, T, want_faces=True, want_bins=False):
        """(q, S, F) with F the total flux at the radial faces (or None); with want_bins
        also the flux of every bin at every face, bin fastest."""
        rho, T = _f64(rho).ravel(), _f64(T).ravel()
        q = np.empty(self.n); S = np.empty(self.n)
        nr, nt, npp = self.shape
        F = np.empty((nr + 1) * nt * npp) if want_faces else None
        Fnu = np.empty((nr + 1) * nt * npp * self.op.nnu) if want_bins else None
        self.L.og_raytrace(C.byref(self.g), C.byref(self.op), C.byref(self.st), _p(rho), _p(T),
                          _p(q), _p(S), _p(F), _p(Fnu))
        return (q, S, F, Fnu) if want_bins else (q, S, F)

    def energy(self, T, S):
        T, S = _f64(T).ravel(), _f64(S).ravel()
        E = np.empty(self.n)
        self.L.og_energy(C.byref(self.g), C.byref(self.op), C.byref(self.fld), _p(T), _p(S), _p(E))
        return E

    def assemble(self, rho, T, En, q, Q=None):
        args = [_f64(x).ravel() for x in (rho, T, En, q)]
        Qa = None if Q is None else _f64(Q).ravel()
        n = self.n
        out = dict(w=np.empty(3 * n), d=np.empty(n), b=np.empty(n), s=np.empty(n),
                   ahat=np.empty(3 * n), bhat=np.empty(n))
        self.L.og_assemble(C.byref(self.g), C.byref(self.op), C.byref(self.fld),
                          *[_p(a) for a in args], _p(Qa), _p(out["w"]), _p(out["d"]),
                          _p(out["b"]), _p(out["s"]), _p(out["ahat"]), _p(out["bhat"]))
        return out

    def spmv(self, ahat, x):
        ahat, x = _f64(ahat).ravel(), _f64(x).ravel()
        y = np.empty(self.n)
        self.L.og_spmv(C.byref(self.g), _p(ahat), _p(x), _p(y))
        return y

    def relres(self, ahat, bhat, y):
        return self.L.og_relres(C.byref(self.g), _p(_f64(ahat).ravel()), _p(_f64(bhat).ravel()),
                               _p(_f64(y).ravel()))

    def cg(self, ahat, bhat, y0, tol, max_iter):
        ahat, bhat = _f64(ahat).ravel(), _f64(bhat).ravel()
        y = _f64(y0).ravel().copy()
        it = C.c_int(0); rr = C.c_double(0)
        st = self.L.og_cg(C.byref(self.g), _p(ahat), _p(bhat), _p(y), tol, max_iter,
                         C.byref(it), C.byref(rr))
        return y, st, it.value, rr.value

    def gmres(self, ahat, bhat, y0, m, tol, max_iter):
        """Restarted GMRES(m); returns (y, status, inner iterations, relative residual)."""
        ahat, bhat = _f64(ahat).ravel(), _f64(bhat).ravel()
        y = _f64(y0).ravel().copy()
        it = C.c_int(0); rr = C.c_double(0)
        st = self.L.og_gmres(C.byref(self.g), _p(ahat), _p(bhat), _p(y), int(m), tol, max_iter,
                            C.byref(it), C.byref(rr))
        return y, st, it.value, rr.value

    def dense_solve(self, ahat, bhat):
        ahat, bhat = _f64(ahat).ravel(), _f64(bhat).ravel()
        y = np.empty(self.n)
        st = self.L.og_dense_solve(C.byref(self.g), _p(ahat), _p(bhat), _p(y))
        if st != 0:
            raise RuntimeError(f"dense solve failed ({st})")
        return y

    def newton(self, E, S, T_start):
        E, S = _f64(E).ravel(), _f64(S).ravel()
        T = _f64(T_start).ravel().copy()
        self.L.og_newton(C.byref(self.g), C.byref(self.op), _p(E), _p(S), _p(T))
        return T

    def force(self, rho, T, w, E, q):
        out = np.empty(4 * self.n)
        args = [_f64(x).ravel() for x in (rho, T, w, E, q)]
        self.L.og_force(C.byref(self.g), C.byref(self.op), C.byref(self.fld),
                       *[_p(a) for a in args], _p(out))
        return out

    def step(self, rho, T, tol=1e-10, max_iter=100000, dense=False, want_force=True, no_fld=False):
        rho = _f64(rho).ravel()
        T = _f64(T).ravel().copy()
        E = np.empty(self.n)
        f = np.empty(4 * self.n) if want_force else None
        it = C.c_int(0); rr = C.c_double(0)
        st = self.L.og_step(C.byref(self.g), C.byref(self.op), C.byref(self.st), C.byref(self.fld),
                           _p(rho), _p(T), _p(E), _p(f), tol, max_iter, 2 if no_fld else int(dense),
                           C.byref(it), C.byref(rr))
        return dict(T=T, E=E, force=f, status=st, iters=it.value, relres=rr.value)

    def relax(self, rho, T, mode="cg", tol=1e-10, max_iter=100000, max_steps=1000, tol_change=1e-4):
        """Steps until the largest relative temperature change is below tol_change.
        mode: "cg", "dense" or "none" (no diffusion).  Returns (T, E, steps, last change)."""
        m = {"cg": 0, "dense": 1, "none": 2}[mode]
        rho = _f64(rho).ravel()
        T = _f64(T).ravel().copy()
        E = np.empty(self.n)
        ch = C.c_double(0)
        k = self.L.og_relax(C.byref(self.g), C.byref(self.op), C.byref(self.st), C.byref(self.fld), _p(rho),
                           _p(T), _p(E), m, tol, max_iter, max_steps, tol_change, C.byref(ch))
        return T, E, k, ch.value

    def tau_rosseland(self, rho, T):
        """Inward Rosseland optical depth at the radial faces ((N_r + 1) per column, 0 at r_out)."""
        rho, T = _f64(rho).ravel(), _f64(T).ravel()
        nr, nt, npp = self.shape
        tau = np.empty((nr + 1) * nt * npp)
        self.L.og_tau_rosseland(C.byref(self.g), C.byref(self.op), _p(rho), _p(T), _p(tau))
        return tau

    def gray_table(self, F):
        """(kappa_gray[n_T], sum F): the one-bin opacity table of gray irradiation."""
        F = _f64(F).ravel()
        kg = np.empty(len(self._keep[3]))
        Fs = self.L.og_gray_table(C.byref(self.op), _p(F), _p(kg))
        return kg, Fs

    # --- table lookups (for pins) ----------------------------------------
    def kappa_nu(self, T, b):
        return self.L.og_kappa_nu(C.byref(self.op), float(T), int(b))

    def kappa_P(self, T):
        return self.L.og_kappa_P(C.byref(self.op), float(T))

    def kappa_R(self, T):
        return self.L.og_kappa_R(C.byref(self.op), float(T))


def star_bins(T_star, nu):
    nu = _f64(nu)
    F = np.empty(len(nu))
    st = lib().og_star_bins(float(T_star), len(nu), _p(nu), _p(F))
    if st != 0:
        raise ValueError("bad star parameters")
    return F


def const_a():
    return lib().og_const_a()


def const_c():
    return lib().og_const_c()


# ----------------------------------------------------------------- network oracle

class NN:
    """Float64 oracle of the U-Net (channels-last tensors, numpy float64)."""

    @staticmethod
    def conv_fwd(shape, x, cin, w, b, cout, relu):
        nr, nt, npp = shape
        x = _f64(x).ravel(); w = _f64(w).ravel()
        b = None if b is None else _f64(b).ravel()
        y = np.empty(nr * nt * npp * cout)
        lib().ognn_conv_fwd(nr, nt, npp, _p(x), cin, _p(w), _p(b), cout, int(relu), _p(y))
        return y

    @staticmethod
    def conv_bwd_data(shape, dy, cout, w, cin):
        nr, nt, npp = shape
        dy = _f64(dy).ravel(); w = _f64(w).ravel()
        dx = np.empty(nr * nt * npp * cin)
        lib().ognn_conv_bwd_data(nr, nt, npp, _p(dy), cout, _p(w), cin, _p(dx))
        return dx

    @staticmethod
    def conv_bwd_weight(shape, x, cin, dy, cout):
        nr, nt, npp = shape
        x = _f64(x).ravel(); dy = _f64(dy).ravel()
        dw = np.empty(27 * cout * cin); db = np.empty(cout)
        lib().ognn_conv_bwd_weight(nr, nt, npp, _p(x), cin, _p(dy), cout, _p(dw), _p(db))
        return dw, db

    @staticmethod
    def pool(shape, x, C):
        nr, nt, npp = shape
        x = _f64(x).ravel()
        y = np.empty((nr // 2) * (nt // 2) * (npp // 2) * C)
        lib().ognn_pool(nr, nt, npp, _p(x), C, _p(y))
        return y

    @staticmethod
    def up(shape, xc, C):
        nr, nt, npp = shape
        xc = _f64(xc).ravel()
        y = np.empty(nr * nt * npp * C)
        lib().ognn_up(nr, nt, npp, _p(xc), C, _p(y))
        return y

    @staticmethod
    def param_count():
        return lib().ognn_param_count()

    @staticmethod
    def param_offset(layer):
        return lib().ognn_param_offset(layer)

    @staticmethod
    def layer_shapes():
        L = lib()
        return [(L.ognn_taps(l), L.ognn_cout(l), L.ognn_cin(l)) for l in range(11)]

    @staticmethod
    def forward_bf16(shape, params, X):
        """U-Net forward with every activation stored as bf16 (ties to even), fp64
        arithmetic otherwise: the network as the matrix-core kernels evaluate it."""
        nr, nt, npp = shape
        params = _f64(params).ravel(); X = _f64(X).ravel()
        z = np.empty(nr * nt * npp)
        lib().ognn_forward_bf16(nr, nt, npp, _p(params), _p(X), _p(z))
        return z

    @staticmethod
    def bf16_round(x):
        return lib().ognn_bf16_round(float(x))

    @staticmethod
    def loss_grad(shape, params, X, e):
        nr, nt, npp = shape
        params = _f64(params).ravel(); X = _f64(X).ravel(); e = _f64(e).ravel()
        grad = np.empty_like(params); z = np.empty(nr * nt * npp)
        L = lib().ognn_loss_grad(nr, nt, npp, _p(params), _p(X), _p(e), _p(grad), _p(z))
        return L, grad, z

    @staticmethod
    def loss_grad_resid(shape, params, X, r, ahat):
        """Residual loss ||A z - r||^2 / ||r||^2 of z = U-Net(X) and its gradient."""
        nr, nt, npp = shape
        params = _f64(params).ravel(); X = _f64(X).ravel(); r = _f64(r).ravel(); ahat = _f64(ahat).ravel()
        grad = np.empty_like(params); z = np.empty(nr * nt * npp)
        L = lib().ognn_loss_grad_resid(nr, nt, npp, _p(params), _p(X), _p(r), _p(ahat), _p(grad), _p(z))
        return L, grad, z

    @staticmethod
    def adam(p, g, m, v, lr, b1, b2, eps, t):
        p = _f64(p).copy(); m = _f64(m).copy(); v = _f64(v).copy(); g = _f64(g)
        lib().ognn_adam(len(p), _p(p), _p(g), _p(m), _p(v), lr, b1, b2, eps, int(t))
        return p, m, v
