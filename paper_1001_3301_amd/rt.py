"""ctypes binding of librtmi (include/rt.h): argument marshalling only.

Every step of the radiation step runs in the HIP library; this module checks tensor
arguments (device, dtype, size, contiguity), passes their device pointers, and turns
non-zero rt_status codes into RtError.  torch provides device memory and the stream.
If librtmi.so is missing, loading fails loudly (build it with
`python -m paper_1001_3301_amd.build`).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtmi.so")

RT_OK, RT_EINVAL, RT_EDEVICE, RT_ENOMEM, RT_ENONFINITE, RT_ENOCONV = range(6)
STATUS_NAMES = {0: "RT_OK", 1: "RT_EINVAL", 2: "RT_EDEVICE", 3: "RT_ENOMEM", 4: "RT_ENONFINITE",
                5: "RT_ENOCONV"}
MODE_FP64, MODE_MIXED, MODE_LEARNED, MODE_GMRES, MODE_NONE = 0, 1, 2, 3, 4
LAUNCH_AUTO, LAUNCH_DIRECT, LAUNCH_GRAPH, LAUNCH_BLOCK = 0, 1, 2, 3
INNER_FCG, INNER_FGMRES = 0, 1
LANES_BINS, LANES_CELLS = 0, 1
PRECOND_JACOBI, PRECOND_LINE, PRECOND_MG = 0, 1, 2
CYCLE_K, CYCLE_V = 0, 1  # cycle = n >= 2: K-cycle steps on levels 1 .. n

dp = C.POINTER(C.c_double)


class RtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Grid(C.Structure):
    _fields_ = [("nr", C.c_int), ("nt", C.c_int), ("np", C.c_int),
                ("r_face", dp), ("th_face", dp), ("ph_face", dp)]


class Opacity(C.Structure):
    _fields_ = [("n_T", C.c_int), ("n_nu", C.c_int), ("T", dp), ("nu", dp), ("kappa", dp),
                ("kappa_P", dp), ("kappa_R", dp)]


class Star(C.Structure):
    _fields_ = [("R_star", C.c_double), ("T_star", C.c_double), ("F_nu", dp)]


class FldParams(C.Structure):
    _fields_ = [("dt", C.c_double), ("c_V", C.c_double), ("T_bc", C.c_double),
                ("E_floor", C.c_double)]


class System(C.Structure):
    _fields_ = [("n", C.c_long), ("ahat", C.c_void_p), ("ahat32", C.c_void_p), ("s", C.c_void_p),
                ("bhat", C.c_void_p), ("w", C.c_void_p), ("chi", C.c_void_p)]


class MgLevelView(C.Structure):
    _fields_ = [("levels", C.c_int), ("nr", C.c_int), ("nt", C.c_int), ("np", C.c_int), ("n", C.c_long)] + \
        [(f, C.c_void_p) for f in ("dg", "ar", "at", "ap", "w", "im", "cp", "q", "g", "rho", "kap")]


class SolveOpts(C.Structure):
    _fields_ = [("mode", C.c_int), ("tol", C.c_double), ("max_iter", C.c_int),
                ("check_every", C.c_int), ("inner_tol", C.c_double), ("inner_max_iter", C.c_int),
                ("net", C.c_void_p), ("restart", C.c_int), ("reduce", C.c_int), ("precond", C.c_int),
                ("launch", C.c_int), ("inner", C.c_int), ("cycle", C.c_int)]


class SolveStats(C.Structure):
    _fields_ = [("status", C.c_int), ("iters", C.c_int), ("outer_iters", C.c_int),
                ("precond_applies", C.c_int), ("fallback", C.c_int), ("relres", C.c_double),
                ("ms", C.c_double), ("ms_dir", C.c_double), ("ms_upd", C.c_double),
                ("kernel_samples", C.c_int), ("reduced", C.c_int), ("ms_black", C.c_double),
                ("handover", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class StepStats(C.Structure):
    _fields_ = [("solve", SolveStats), ("ms_raytrace", C.c_double), ("ms_assemble", C.c_double),
                ("ms_solve", C.c_double), ("ms_newton", C.c_double), ("ms_total", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "solve"}
        d["solve"] = self.solve.as_dict()
        return d


class RelaxStats(C.Structure):
    _fields_ = [("steps", C.c_int), ("last_change", C.c_double), ("krylov_iters", C.c_long),
                ("ms", C.c_double), ("ms_device", C.c_double), ("last", StepStats)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "last"}
        d["last"] = self.last.as_dict()
        return d


# Every symbol include/rt.h declares (checked by the tests).
EXPORTS = ["rt_create", "rt_destroy", "rt_last_error", "rt_ncell", "rt_star_bin_flux",
           "rt_set_opacity", "rt_set_star", "rt_raytrace", "rt_raytrace_mapped", "rt_energy", "rt_fld_assemble",
           "rt_spmv", "rt_fld_solve", "rt_temperature", "rt_force", "rt_step", "rt_step_fields",
           "rt_gray_table", "rt_relax", "rt_rosseland_depth", "rt_precond_apply", "rt_mg_apply", "rt_mg_level",
           "rt_net_create", "rt_net_destroy", "rt_net_last_error", "rt_net_param_count",
           "rt_net_get_params", "rt_net_get_grads", "rt_net_set_params", "rt_net_save", "rt_net_load",
           "rt_net_forward", "rt_net_apply", "rt_net_loss_grad", "rt_net_loss_grad_resid", "rt_net_adam", "rt_dataset_create",
           "rt_dataset_destroy", "rt_dataset_size", "rt_dataset_add", "rt_dataset_add_learned", "rt_net_train",
           "rt_nn_conv3d_fwd", "rt_nn_conv3d_fwd_pool", "rt_nn_conv3d_bwd_data", "rt_nn_conv3d_bwd_weight",
           "rt_nn_conv3d_bwd_weight_noalloc"]


LOSS_ERROR, LOSS_RESIDUAL = 0, 1


class NetConfig(C.Structure):
    _fields_ = [("seed", C.c_uint)]


class TrainOpts(C.Structure):
    _fields_ = [("epochs", C.c_int), ("lr", C.c_double), ("seed", C.c_uint), ("loss", C.c_int)]


class TrainStats(C.Structure):
    _fields_ = [("steps", C.c_int), ("loss_first_epoch", C.c_double), ("loss_last_epoch", C.c_double),
                ("ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}

_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1001_3301_amd.build`")
    L = C.CDLL(LIB_PATH)
    P, vp = C.POINTER, C.c_void_p
    L.rt_create.argtypes = [P(vp), P(Grid), C.c_int, vp]
    L.rt_destroy.argtypes = [vp]
    L.rt_destroy.restype = None
    L.rt_last_error.argtypes = [vp]
    L.rt_last_error.restype = C.c_char_p
    L.rt_ncell.argtypes = [vp]
    L.rt_ncell.restype = C.c_long
    L.rt_star_bin_flux.argtypes = [C.c_double, C.c_int, dp, dp]
    L.rt_set_opacity.argtypes = [vp, P(Opacity)]
    L.rt_set_star.argtypes = [vp, P(Star)]
    L.rt_raytrace.argtypes = [vp, P(Opacity), P(Star), vp, vp, vp, vp, vp, vp]
    L.rt_raytrace_mapped.argtypes = [vp, C.c_int, vp, vp, vp, vp]
    L.rt_energy.argtypes = [vp, P(Opacity), P(FldParams), vp, vp, vp]
    L.rt_fld_assemble.argtypes = [vp, P(Opacity), P(FldParams), vp, vp, vp, vp, vp, P(System)]
    L.rt_spmv.argtypes = [vp, vp, vp]
    L.rt_fld_solve.argtypes = [vp, P(SolveOpts), vp, P(SolveStats)]
    L.rt_temperature.argtypes = [vp, P(Opacity), vp, vp, vp]
    L.rt_force.argtypes = [vp, vp, vp, vp]
    L.rt_step.argtypes = [vp, P(Opacity), P(Star), P(FldParams), P(SolveOpts), vp, vp, vp, vp,
                          P(StepStats)]
    L.rt_step_fields.argtypes = [vp, P(vp), P(vp), P(vp)]
    L.rt_gray_table.argtypes = [P(Opacity), dp, dp, dp, dp]
    L.rt_rosseland_depth.argtypes = [vp, P(Opacity), vp, vp, vp]
    L.rt_precond_apply.argtypes = [vp, vp, vp]
    L.rt_mg_apply.argtypes = [vp, vp, vp]
    L.rt_mg_level.argtypes = [vp, C.c_int, C.POINTER(MgLevelView)]
    L.rt_relax.argtypes = [vp, P(Opacity), P(Star), P(FldParams), P(SolveOpts), vp, vp, vp, C.c_double,
                           C.c_int, P(RelaxStats)]
    fp = P(C.c_float)
    L.rt_net_create.argtypes = [P(NetConfig), P(vp)]
    L.rt_net_destroy.argtypes = [vp]
    L.rt_net_destroy.restype = None
    L.rt_net_last_error.argtypes = [vp]
    L.rt_net_last_error.restype = C.c_char_p
    L.rt_net_param_count.argtypes = [vp]
    L.rt_net_param_count.restype = C.c_long
    L.rt_net_get_params.argtypes = [vp, fp, C.c_long]
    L.rt_net_get_grads.argtypes = [vp, fp, C.c_long]
    L.rt_net_set_params.argtypes = [vp, fp, C.c_long]
    L.rt_net_save.argtypes = [vp, C.c_char_p]
    L.rt_net_load.argtypes = [vp, C.c_char_p]
    L.rt_net_forward.argtypes = [vp, vp, vp, vp]
    L.rt_net_apply.argtypes = [vp, vp, vp, vp]
    L.rt_net_loss_grad.argtypes = [vp, vp, vp, vp, vp, P(C.c_double)]
    L.rt_net_loss_grad_resid.argtypes = [vp, vp, vp, vp, vp, vp, P(C.c_double)]
    L.rt_net_adam.argtypes = [vp, vp, C.c_double]
    L.rt_dataset_create.argtypes = [vp, C.c_int, P(vp)]
    L.rt_dataset_destroy.argtypes = [vp]
    L.rt_dataset_destroy.restype = None
    L.rt_dataset_size.argtypes = [vp]
    L.rt_dataset_add.argtypes = [vp, vp, vp, P(C.c_int), C.c_int]
    L.rt_dataset_add_learned.argtypes = [vp, vp, vp, vp, P(C.c_int), C.c_int]
    L.rt_net_train.argtypes = [vp, vp, vp, P(TrainOpts), P(TrainStats)]
    ip = C.c_int
    L.rt_nn_conv3d_fwd.argtypes = [vp, ip, ip, ip, vp, ip, ip, vp, ip, vp, vp, ip, ip, vp, vp]
    L.rt_nn_conv3d_fwd_pool.argtypes = [vp, ip, ip, ip, vp, vp, vp, vp, vp]
    L.rt_nn_conv3d_bwd_data.argtypes = [vp, ip, ip, ip, vp, vp, ip, vp, ip, vp, ip, vp]
    L.rt_nn_conv3d_bwd_weight.argtypes = [vp, ip, ip, ip, vp, vp, ip, vp, ip, ip, vp, ip, vp, vp]
    L.rt_nn_conv3d_bwd_weight_noalloc.argtypes = [vp, ip, ip, ip, vp, vp, ip, vp, ip, ip, vp, ip, vp, vp]
    _lib = L
    return L


def _host(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _hp(a):
    return a.ctypes.data_as(dp)


def star_bin_flux(T_star: float, nu) -> np.ndarray:
    """Eq. (20) bin fluxes (host computation in the library)."""
    nu = _host(nu)
    out = np.empty_like(nu)
    st = lib().rt_star_bin_flux(float(T_star), len(nu), _hp(nu), _hp(out))
    if st != RT_OK:
        raise RtError(st, lib().rt_last_error(None).decode())
    return out


def gray_table(op, F_nu):
    """Eqs. (18)-(19) as a one-bin table (host computation in the library): returns
    (kappa_gray[n_T], F_total, nu_gray)."""
    arrs = [_host(op.T), _host(op.nu), _host(op.kappa), _host(op.kappa_P), _host(op.kappa_R)]
    o = Opacity(len(arrs[0]), len(arrs[1]), *[_hp(a) for a in arrs])
    F = _host(F_nu)
    kg = np.empty(len(arrs[0]))
    Ft, nug = C.c_double(), C.c_double()
    st = lib().rt_gray_table(C.byref(o), _hp(F), _hp(kg), C.byref(Ft), C.byref(nug))
    if st != RT_OK:
        raise RtError(st, lib().rt_last_error(None).decode())
    return kg, Ft.value, nug.value


class GrayOpacity:
    """The one-bin table of a gray run (same temperatures and mean opacities)."""

    def __init__(self, op, kappa_gray, nu_gray):
        self.T, self.kappa_P, self.kappa_R = op.T, op.kappa_P, op.kappa_R
        self.kappa = np.asarray(kappa_gray, dtype=np.float64).reshape(-1, 1)
        self.nu = np.array([nu_gray])


def solve_opts(mode=MODE_FP64, tol=1e-8, max_iter=100000, check_every=32, inner_tol=1e-4,
               inner_max_iter=0, net=None, restart=30, reduce=0, precond=0, launch=0, inner=INNER_FCG,
               cycle=CYCLE_K) -> SolveOpts:
    nh = None if net is None else (net.h if isinstance(net, Net) else net)
    o = SolveOpts(mode, tol, max_iter, check_every, inner_tol, inner_max_iter, nh, restart, int(reduce),
                  int(precond), int(launch), int(inner), int(cycle))
    o._net = net  # keeps the network alive as long as the options refer to it
    return o


class Context:
    """One rt_ctx bound to torch's current stream on the current device."""

    def __init__(self, r_face, th_face, ph_face, n_nu: int, stream=None):
        import torch
        self._torch = torch
        self._faces = [_host(x) for x in (r_face, th_face, ph_face)]
        rf, tf, pf = self._faces
        self.shape = (len(rf) - 1, len(tf) - 1, len(pf) - 1)
        self.n = int(np.prod(self.shape))
        self.n_nu = n_nu
        g = Grid(self.shape[0], self.shape[1], self.shape[2], _hp(rf), _hp(tf), _hp(pf))
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        h = C.c_void_p()
        st = lib().rt_create(C.byref(h), C.byref(g), n_nu, C.c_void_p(stream))
        if st != RT_OK:
            raise RtError(st, lib().rt_last_error(None).decode())
        self.h = h
        self._op = None
        self._star = None
        self._keep = []

    @classmethod
    def from_workload(cls, wl, stream=None, gray=False):
        """Context with the workload's tables; gray=True gives the gray-irradiation run
        (one bin: the flux-weighted table and the total stellar flux)."""
        g = wl.grid
        F = star_bin_flux(wl.T_star, wl.opacity.nu)
        op = wl.opacity
        if gray:
            kg, Ft, nug = gray_table(op, F)
            op, F = GrayOpacity(op, kg, nug), np.array([Ft])
        ctx = cls(g.r_face, g.th_face, g.ph_face, len(op.nu), stream)
        ctx.set_opacity(op)
        ctx.set_star(wl.R_star, wl.T_star, F)
        ctx.params = FldParams(wl.dt, wl.c_V, wl.T_bc, wl.E_floor)
        return ctx

    def close(self):
        if getattr(self, "h", None):
            lib().rt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- helpers -----------------------------------------------------------
    def _chk(self, st):
        if st != RT_OK:
            raise RtError(st, lib().rt_last_error(self.h).decode())

    def _dev(self, t, n, name, dtype=None, allow_none=False):
        torch = self._torch
        if t is None:
            if allow_none:
                return None
            raise ValueError(f"{name} is required")
        dtype = dtype or torch.float64
        if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"{name}: need a contiguous {dtype} CUDA tensor of {n} elements, got "
                             f"{t.dtype} {tuple(t.shape)} on {t.device}")
        return C.c_void_p(t.data_ptr())

    def set_opacity(self, op):
        arrs = [_host(op.T), _host(op.nu), _host(op.kappa), _host(op.kappa_P), _host(op.kappa_R)]
        o = Opacity(len(arrs[0]), len(arrs[1]), *[_hp(a) for a in arrs])
        self._chk(lib().rt_set_opacity(self.h, C.byref(o)))
        self._op = (o, arrs)

    def set_star(self, R_star, T_star, F_nu):
        F = _host(F_nu)
        s = Star(float(R_star), float(T_star), _hp(F))
        self._chk(lib().rt_set_star(self.h, C.byref(s)))
        self._star = (s, F)

    # --- the step's calls --------------------------------------------------
    def raytrace(self, rho, T, q, S, F_face=None, F_face_nu=None):
        """F_face_nu, if given, receives the flux of every bin at every radial face, bin
        fastest ((N_r + 1) N_theta N_phi n_nu values)."""
        nr, nt, npp = self.shape
        nf = (nr + 1) * nt * npp
        args = [self._dev(rho, self.n, "rho"), self._dev(T, self.n, "T"), self._dev(q, self.n, "q"),
                self._dev(S, self.n, "S"),
                self._dev(F_face, nf, "F_face", allow_none=True),
                self._dev(F_face_nu, nf * self.n_nu, "F_face_nu", allow_none=True)]
        self._chk(lib().rt_raytrace(self.h, None, None, *args))

    def raytrace_mapped(self, mapping, rho, T, q, S):
        """q and S of raytrace with lanes on bins (LANES_BINS) or on radial cells (LANES_CELLS)."""
        self._chk(lib().rt_raytrace_mapped(self.h, int(mapping), self._dev(rho, self.n, "rho"),
                                           self._dev(T, self.n, "T"), self._dev(q, self.n, "q"),
                                           self._dev(S, self.n, "S")))

    def energy(self, T, S, E, params=None):
        p = params or self.params
        self._chk(lib().rt_energy(self.h, None, C.byref(p), self._dev(T, self.n, "T"),
                                  self._dev(S, self.n, "S"), self._dev(E, self.n, "E")))

    def assemble(self, rho, T, En, q, Q=None, params=None):
        p = params or self.params
        sysv = System()
        self._chk(lib().rt_fld_assemble(self.h, None, C.byref(p), self._dev(rho, self.n, "rho"),
                                        self._dev(T, self.n, "T"), self._dev(En, self.n, "E_n"),
                                        self._dev(q, self.n, "q"),
                                        self._dev(Q, self.n, "Q", allow_none=True), C.byref(sysv)))
        return sysv

    def system_tensors(self, sysv):
        """Copies of the assembled system (ahat [3n], ahat32 [3n], s, bhat, w [3n], chi)."""
        torch = self._torch
        n = self.n
        out = {}
        for name, cnt, dt in (("ahat", 3 * n, torch.float64), ("ahat32", 3 * n, torch.float32),
                              ("s", n, torch.float64), ("bhat", n, torch.float64),
                              ("w", 3 * n, torch.float64), ("chi", n, torch.float64)):
            t = torch.empty(cnt, dtype=dt, device="cuda")
            _memcpy_d2d(t.data_ptr(), getattr(sysv, name), t.numel() * t.element_size())
            out[name] = t
        return out

    def spmv(self, x, y):
        self._chk(lib().rt_spmv(self.h, self._dev(x, self.n, "x"), self._dev(y, self.n, "y")))

    def solve(self, E, opts: SolveOpts, raise_on_error=True):
        st = SolveStats()
        rc = lib().rt_fld_solve(self.h, C.byref(opts), self._dev(E, self.n, "E"), C.byref(st))
        if raise_on_error:
            self._chk(rc)
        return rc, st.as_dict()

    def temperature(self, E, S, T):
        self._chk(lib().rt_temperature(self.h, None, self._dev(E, self.n, "E"),
                                       self._dev(S, self.n, "S"), self._dev(T, self.n, "T")))

    def force(self, E, q, f):
        self._chk(lib().rt_force(self.h, self._dev(E, self.n, "E"), self._dev(q, self.n, "q"),
                                 self._dev(f, 4 * self.n, "f")))

    def step(self, rho, T, E, opts: SolveOpts, f_rad=None, params=None, raise_on_error=True):
        p = params or self.params
        st = StepStats()
        rc = lib().rt_step(self.h, None, None, C.byref(p), C.byref(opts),
                           self._dev(rho, self.n, "rho"), self._dev(T, self.n, "T"),
                           self._dev(E, self.n, "E"),
                           self._dev(f_rad, 4 * self.n, "f_rad", allow_none=True), C.byref(st))
        if raise_on_error:
            self._chk(rc)
        return rc, st.as_dict()

    def precond_apply(self, r, z):
        """rt_precond_apply: z = M^-1 r, radial-line block Jacobi of the current system."""
        self._chk(lib().rt_precond_apply(self.h, self._dev(r, self.n, "r"), self._dev(z, self.n, "z")))

    def mg_apply(self, r, z):
        """rt_mg_apply: z = M_mg r, one multigrid V-cycle of the current system."""
        self._chk(lib().rt_mg_apply(self.h, self._dev(r, self.n, "r"), self._dev(z, self.n, "z")))

    def mg_level(self, level):
        """rt_mg_level: copies of one level's float32 arrays (None where the view has none)."""
        torch = self._torch
        v = MgLevelView()
        self._chk(lib().rt_mg_level(self.h, int(level), C.byref(v)))
        lines = v.nr * v.nt
        out = dict(levels=v.levels, nr=v.nr, nt=v.nt, np=v.np, n=v.n)
        for f in ("dg", "ar", "at", "ap", "w", "im", "cp", "q", "g", "rho", "kap"):
            ptr = getattr(v, f)
            if not ptr:
                out[f] = None
                continue
            cnt = lines if f in ("rho", "kap") else v.n
            t = torch.empty(cnt, dtype=torch.float32, device="cuda")
            _memcpy_d2d(t.data_ptr(), ptr, cnt * 4)
            out[f] = t
        return out

    def rosseland_depth(self, rho, T, tau):
        """rt_rosseland_depth: inward tau_R at the radial faces ((N_r + 1) per column)."""
        nr, nt, npp = self.shape
        self._chk(lib().rt_rosseland_depth(self.h, None, self._dev(rho, self.n, "rho"), self._dev(T, self.n, "T"),
                                           self._dev(tau, (nr + 1) * nt * npp, "tau")))

    def relax(self, rho, T, E, opts: SolveOpts, tol_change=1e-4, max_steps=10000, params=None,
              raise_on_error=True):
        """rt_relax: main iterations until the largest relative temperature change of a
        step is below tol_change.  Returns (status, stats dict)."""
        p = params or self.params
        st = RelaxStats()
        rc = lib().rt_relax(self.h, None, None, C.byref(p), C.byref(opts), self._dev(rho, self.n, "rho"),
                            self._dev(T, self.n, "T"), self._dev(E, self.n, "E"), float(tol_change),
                            int(max_steps), C.byref(st))
        if raise_on_error:
            self._chk(rc)
        return rc, st.as_dict()

    def step_fields(self):
        """Copies of the last step's q_star, S_abs and E^n."""
        torch = self._torch
        ptrs = [C.c_void_p() for _ in range(3)]
        self._chk(lib().rt_step_fields(self.h, *[C.byref(p) for p in ptrs]))
        out = []
        for p in ptrs:
            t = torch.empty(self.n, dtype=torch.float64, device="cuda")
            _memcpy_d2d(t.data_ptr(), p.value, t.numel() * 8)
            out.append(t)
        return out


class Net:
    """The learned preconditioner's network (rt_net)."""

    def __init__(self, seed=1):
        h = C.c_void_p()
        cfg = NetConfig(seed)
        st = lib().rt_net_create(C.byref(cfg), C.byref(h))
        if st != RT_OK:
            raise RtError(st, lib().rt_net_last_error(None).decode())
        self.h = h
        self.n = lib().rt_net_param_count(h)

    def _chk(self, st):
        if st != RT_OK:
            raise RtError(st, lib().rt_net_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().rt_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        out = np.empty(self.n, dtype=np.float32)
        self._chk(lib().rt_net_get_params(self.h, out.ctypes.data_as(C.POINTER(C.c_float)), self.n))
        return out

    def get_grads(self):
        out = np.empty(self.n, dtype=np.float32)
        self._chk(lib().rt_net_get_grads(self.h, out.ctypes.data_as(C.POINTER(C.c_float)), self.n))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        self._chk(lib().rt_net_set_params(self.h, p.ctypes.data_as(C.POINTER(C.c_float)), len(p)))

    def save(self, path):
        self._chk(lib().rt_net_save(self.h, str(path).encode()))

    def load(self, path):
        self._chk(lib().rt_net_load(self.h, str(path).encode()))

    def forward(self, ctx, X, z):
        self._chk(lib().rt_net_forward(ctx.h, self.h, ctx._dev(X, ctx.n * 16, "X", ctx._torch.bfloat16),
                                       ctx._dev(z, ctx.n, "z", ctx._torch.float32)))

    def apply(self, ctx, r, z):
        """z = M(r), the preconditioner's action on the fp32 residual r on ctx's system."""
        self._chk(lib().rt_net_apply(ctx.h, self.h, ctx._dev(r, ctx.n, "r", ctx._torch.float32),
                                     ctx._dev(z, ctx.n, "z", ctx._torch.float32)))

    def loss_grad(self, ctx, X, e, z=None):
        L = C.c_double()
        self._chk(lib().rt_net_loss_grad(ctx.h, self.h, ctx._dev(X, ctx.n * 16, "X", ctx._torch.bfloat16),
                                         ctx._dev(e, ctx.n, "e", ctx._torch.float32),
                                         ctx._dev(z, ctx.n, "z", ctx._torch.float32, allow_none=True),
                                         C.byref(L)))
        return L.value

    def loss_grad_resid(self, ctx, X, r, a32, z=None):
        """Residual loss ||A z - r||^2 / ||r||^2 (a32: the scaled operator, 3n fp32) and
        the backward pass."""
        L = C.c_double()
        self._chk(lib().rt_net_loss_grad_resid(ctx.h, self.h, ctx._dev(X, ctx.n * 16, "X", ctx._torch.bfloat16),
                                               ctx._dev(r, ctx.n, "r", ctx._torch.float32),
                                               ctx._dev(a32, 3 * ctx.n, "a32", ctx._torch.float32),
                                               ctx._dev(z, ctx.n, "z", ctx._torch.float32, allow_none=True),
                                               C.byref(L)))
        return L.value

    def adam(self, ctx, lr):
        self._chk(lib().rt_net_adam(ctx.h, self.h, float(lr)))

    def train(self, ctx, ds, epochs, lr, seed=0, loss=0):
        """loss: LOSS_ERROR (||z - e||^2 / ||e||^2) or LOSS_RESIDUAL (||A z - r||^2 / ||r||^2)."""
        o = TrainOpts(epochs, lr, seed, int(loss))
        st = TrainStats()
        self._chk(lib().rt_net_train(ctx.h, self.h, ds.h, C.byref(o), C.byref(st)))
        return st.as_dict()


class Dataset:
    """(residual -> error) training pairs made by the float64 method on a context's grid."""

    def __init__(self, ctx, capacity):
        h = C.c_void_p()
        st = lib().rt_dataset_create(ctx.h, int(capacity), C.byref(h))
        if st != RT_OK:
            raise RtError(st, lib().rt_net_last_error(None).decode())
        self.h = h
        self.ctx = ctx

    def close(self):
        if getattr(self, "h", None):
            lib().rt_dataset_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return lib().rt_dataset_size(self.h)

    def add(self, E0, iters):
        it = (C.c_int * len(iters))(*iters)
        st = lib().rt_dataset_add(self.ctx.h, self.h, self.ctx._dev(E0, self.ctx.n, "E0"), it, len(iters))
        if st != RT_OK:
            raise RtError(st, lib().rt_net_last_error(None).decode())

    def add_learned(self, net, E0, iters):
        """Pairs from the residuals of k learned flexible-CG iterations with `net`."""
        it = (C.c_int * len(iters))(*iters)
        st = lib().rt_dataset_add_learned(self.ctx.h, self.h, net.h, self.ctx._dev(E0, self.ctx.n, "E0"), it,
                                          len(iters))
        if st != RT_OK:
            raise RtError(st, lib().rt_net_last_error(None).decode())


def _vp(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def nn_conv_fwd(shape, x1, c1, up1, x2, c2, w, b, cout, relu, y=None, yf=None):
    """Layer-level forward convolution (device tensors; bf16 x1 / x2 / w, fp32 b / yf)."""
    import torch
    nr, nt, npp = shape
    st = lib().rt_nn_conv3d_fwd(C.c_void_p(torch.cuda.current_stream().cuda_stream), nr, nt, npp, _vp(x1), c1,
                                int(up1), _vp(x2), c2, _vp(w), _vp(b), cout, int(relu), _vp(y), _vp(yf))
    if st != RT_OK:
        raise RtError(st, lib().rt_net_last_error(None).decode())


def nn_conv_fwd_pool(shape, x, w, b, y, yp):
    """16 -> 16 forward convolution with ReLU and its 2x2x2 average pool in one pass."""
    import torch
    nr, nt, npp = shape
    st = lib().rt_nn_conv3d_fwd_pool(C.c_void_p(torch.cuda.current_stream().cuda_stream), nr, nt, npp, _vp(x),
                                     _vp(w), _vp(b), _vp(y), _vp(yp))
    if st != RT_OK:
        raise RtError(st, lib().rt_net_last_error(None).decode())


def nn_conv_bwd_data(shape, dy, yrelu, cout, wt, c1, d1, c2=0, d2=None):
    import torch
    nr, nt, npp = shape
    st = lib().rt_nn_conv3d_bwd_data(C.c_void_p(torch.cuda.current_stream().cuda_stream), nr, nt, npp, _vp(dy),
                                     _vp(yrelu), cout, _vp(wt), c1, _vp(d1), c2, _vp(d2))
    if st != RT_OK:
        raise RtError(st, lib().rt_net_last_error(None).decode())


def nn_conv_bwd_weight(shape, dy, yrelu, cout, x1, c1, up1, x2, c2, dw, db, noalloc=False):
    """rt_nn_conv3d_bwd_weight, or (noalloc=True) its allocation-free variant, which only
    enqueues on torch's current stream."""
    import torch
    nr, nt, npp = shape
    fn = lib().rt_nn_conv3d_bwd_weight_noalloc if noalloc else lib().rt_nn_conv3d_bwd_weight
    st = fn(C.c_void_p(torch.cuda.current_stream().cuda_stream), nr, nt, npp, _vp(dy), _vp(yrelu), cout, _vp(x1),
            c1, int(up1), _vp(x2), c2, _vp(dw), _vp(db))
    if st != RT_OK:
        raise RtError(st, lib().rt_net_last_error(None).decode())


_hip = None


def _memcpy_d2d(dst: int, src: int, nbytes: int):
    """Device-to-device copy through the HIP runtime (synchronises the device first)."""
    global _hip
    import torch
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip.hipDeviceSynchronize.argtypes = []
    torch.cuda.synchronize()
    rc = _hip.hipMemcpy(C.c_void_p(dst), C.c_void_p(src), C.c_size_t(nbytes), 3)  # device to device
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")
    torch.cuda.synchronize()
