"""Test-side reference of the multigrid preconditioner (numpy, array form).

The solver's multigrid preconditioner is not part of the paper (the paper preconditions
its Krylov solve by block Jacobi); the answer it helps reach is the solution of the
scaled FLD system, which the oracle checks.  This module re-derives the preconditioner
itself, independently of the HIP code, so that its pieces can be compared one by one:

* levels: the scaled 7-point operator A_0 = A^ (unit diagonal, couplings ar / at / ap
  to the +r / +theta / +phi neighbour, periodic in phi), and below it Galerkin operators
  A_(l+1) = P_l^T A_l P_l for aggregates of 1 x 2 x 2 cells (radius kept, theta and phi
  pairs merged; a lone last row where a size is odd), with P_l[f, C] = B_f / Bc_C, B_0 =
  1/s (so the unscaled operator's constants lie in every coarse space) and Bc_C^2 the
  sum of B_f^2 over the aggregate.  Coarsening stops at a single radial line.
* smoother: damped block Jacobi on phi lines (the diagonal and phi couplings of each
  (r, theta) line, periodic), x <- x + omega M^-1 (b - A x).
* cycle: pre-smoothing from zero, the residual restricted by P^T, the coarse
  correction, prolonged by P, post-smoothing; the coarsest line is solved exactly.  The
  coarse correction of levels 1 to 3 (the K levels, when not the last) is two steps of
  flexible CG on that level preconditioned by the cycle from it (Notay's K-cycle):
  x = a1 p1 + a2 p2, p1 = z1, p2 = z2 + beta p1, beta = -(z2.q1)/(p1.q1), q = A p,
  a = (p.r)/(p.q); elsewhere the cycle one level down (a V-cycle).

Arrays are (n_phi, n_theta, n_r), r fastest, as the device layout.
"""
import numpy as np


def _pair_sum(a, axis, f):
    """Sum neighbouring pairs along `axis` (f = 2), padding an odd length with zeros."""
    if f == 1:
        return a.copy()
    n = a.shape[axis]
    if n % 2:
        pad = [(0, 0)] * a.ndim
        pad[axis] = (0, 1)
        a = np.pad(a, pad)
    sh = list(a.shape)
    sh[axis:axis + 1] = [sh[axis] // 2, 2]
    return a.reshape(sh).sum(axis=axis + 1)


def _up(a, axis, f, n):
    """Repeat each coarse entry over its f children along `axis` (length n)."""
    if f == 1:
        return a
    return np.repeat(a, 2, axis=axis).take(np.arange(n), axis=axis)


def spmv(lv, x):
    dg, ar, at, ap = lv["dg"], lv["ar"], lv["at"], lv["ap"]
    y = dg * x
    y[:, :, :-1] += ar[:, :, :-1] * x[:, :, 1:]
    y[:, :, 1:] += ar[:, :, :-1] * x[:, :, :-1]
    y[:, :-1, :] += at[:, :-1, :] * x[:, 1:, :]
    y[:, 1:, :] += at[:, :-1, :] * x[:, :-1, :]
    if x.shape[0] > 1:
        y += ap * np.roll(x, -1, axis=0) + np.roll(ap * x, 1, axis=0)
    return y


def coarsen(lv):
    """The next level (Galerkin operator, near-null vector) and the weights w = B / Bc."""
    dg, ar, at, ap, B = lv["dg"], lv["ar"], lv["at"], lv["ap"], lv["B"]
    npf, ntf, nr = dg.shape
    ft, fp = (2 if ntf > 1 else 1), (2 if npf > 1 else 1)

    def agg(a):
        return _pair_sum(_pair_sum(a, 1, ft), 0, fp)

    def up(a):
        return _up(_up(a, 1, ft, ntf), 0, fp, npf)

    Bc = np.sqrt(agg(B * B))
    w = B / up(Bc)
    # internal couplings: theta pairs (2J, 2J+1), phi pairs (2K, 2K+1), and for two phi
    # cells merged into one, the periodic coupling between them as well
    it = np.zeros_like(dg)
    if ft == 2:
        it[:, 0:ntf - 1:2, :] = at[:, 0:ntf - 1:2, :] * w[:, 0:ntf - 1:2, :] * w[:, 1:ntf:2, :]
    ip = np.zeros_like(dg)
    if fp == 2:
        ip[0:npf - 1:2] = ap[0:npf - 1:2] * w[0:npf - 1:2] * w[1:npf:2]
        if npf == 2:
            ip[1] = ap[1] * w[1] * w[0]
    dgc = agg(dg * w * w + 2.0 * (it + ip))
    arc = agg(np.concatenate([ar[:, :, :-1] * w[:, :, :-1] * w[:, :, 1:], np.zeros_like(ar[:, :, :1])], axis=2))
    # couplings that leave an aggregate towards +theta: from its last child row 2J+1
    atc = np.zeros_like(agg(dg))
    if ft == 2:
        lt = np.zeros_like(dg)
        lt[:, 1:ntf - 1:2, :] = at[:, 1:ntf - 1:2, :] * w[:, 1:ntf - 1:2, :] * w[:, 2:ntf:2, :]
        atc = agg(lt)
    else:
        atc = agg(at * w * np.concatenate([w[:, 1:, :], np.zeros_like(w[:, :1, :])], axis=1))
    npc = (npf + 1) // 2 if fp == 2 else 1
    if fp == 2 and npc >= 2:
        # from the last child k_last = min(2K+1, npf-1) towards (k_last+1) mod npf
        lp = np.zeros_like(dg)
        for K in range(npc):
            kl = min(2 * K + 1, npf - 1)
            lp[kl] = ap[kl] * w[kl] * w[(kl + 1) % npf]
        apc = agg(lp)
    elif fp == 1 and npf > 1:
        apc = agg(ap * w * np.roll(w, -1, axis=0))
    else:
        apc = np.zeros_like(dgc)
    return dict(dg=dgc, ar=arc, at=atc, ap=apc, B=Bc), w


def line_factors(lv):
    """Factors of the periodic phi-line matrices M (Sherman-Morrison on the Thomas
    factorisation of T = M - u v^T, gamma = -dg_0), and q = T^-1 u, g = T^-1 e_0."""
    dg, ap = lv["dg"], lv["ap"]
    m = dg.shape[0]
    im = np.zeros_like(dg); cp = np.zeros_like(dg); q = np.zeros_like(dg); g = np.zeros_like(dg)
    rho = np.zeros_like(dg[0]); kap = np.zeros_like(dg[0])
    if m == 1:
        im[0] = 1.0 / dg[0]
        return dict(im=im, cp=cp, q=q, g=g, rho=rho, kap=kap, e=np.zeros_like(dg))
    e = ap.copy()
    if m == 2:
        e = np.zeros_like(dg); e[0] = ap[0] + ap[1]
        Td = dg.copy()
    else:
        gam = -dg[0]
        Td = dg.copy()
        Td[0] = dg[0] - gam
        Td[m - 1] = dg[m - 1] - ap[m - 1] ** 2 / gam
        rho = ap[m - 1] / gam
    mk = Td[0]
    im[0] = 1.0 / mk
    for k in range(1, m):
        mk = Td[k] - e[k - 1] ** 2 * im[k - 1]
        im[k] = 1.0 / mk
    for k in range(m - 1):
        cp[k] = e[k] * im[k]
    f = dict(im=im, cp=cp, q=q, g=g, rho=rho, kap=kap, e=e)
    if m >= 3:
        u = np.zeros_like(dg); u[0] = -dg[0]; u[m - 1] = ap[m - 1]
        e0 = np.zeros_like(dg); e0[0] = 1.0
        f["q"] = _thomas(f, u)
        f["g"] = _thomas(f, e0)
        f["kap"] = 1.0 / (1.0 + f["q"][0] + rho * f["q"][m - 1])
    return f


def _thomas(f, rhs):
    im, cp, e = f["im"], f["cp"], f["e"]
    m = rhs.shape[0]
    d = np.zeros_like(rhs)
    d[0] = rhs[0] * im[0]
    for k in range(1, m):
        d[k] = (rhs[k] - e[k - 1] * d[k - 1]) * im[k]
    y = np.zeros_like(rhs)
    y[m - 1] = d[m - 1]
    for k in range(m - 2, -1, -1):
        y[k] = d[k] - cp[k] * y[k + 1]
    return y


def line_solve(f, rhs):
    """M^-1 rhs on every phi line."""
    y = _thomas(f, rhs)
    m = rhs.shape[0]
    if m >= 3:
        fac = f["kap"] * (y[0] + f["rho"] * y[m - 1])
        y = y - fac * f["q"]
    return y


def radial_solve(lv, b):
    """Exact solve on a level that is a single radial line (tridiagonal in r)."""
    dg, ar = lv["dg"][0, 0], lv["ar"][0, 0]
    n = dg.shape[0]
    A = np.diag(dg) + np.diag(ar[:-1], 1) + np.diag(ar[:-1], -1)
    return np.linalg.solve(A, b[0, 0]).reshape(b.shape)


class Hierarchy:
    def __init__(self, shape, ahat, s, omega=0.8, dtype=np.float64, klevels=(1, 2, 3)):
        nr, nt, nph = shape
        n = nr * nt * nph
        a = np.asarray(ahat, dtype=np.float64).reshape(3, nph, nt, nr)
        lv = dict(dg=np.ones((nph, nt, nr)), ar=a[0].copy(), at=a[1].copy(), ap=a[2].copy(),
                  B=(1.0 / np.asarray(s, dtype=np.float64)).reshape(nph, nt, nr))
        self.levels, self.w, self.f = [], [], []
        while True:
            self.levels.append(lv)
            if lv["dg"].shape[0] * lv["dg"].shape[1] == 1:
                break
            self.f.append(line_factors(lv))
            lv, w = coarsen(lv)
            self.w.append(w)
        self.omega = omega
        self.dtype = dtype
        self.klevels = tuple(l for l in klevels if 0 < l < len(self.levels) - 1)
        if dtype != np.float64:
            cast = lambda d: {k: (v.astype(dtype) if isinstance(v, np.ndarray) else v) for k, v in d.items()}
            self.levels = [cast(l) for l in self.levels]
            self.f = [cast(f) for f in self.f]
            self.w = [w.astype(dtype) for w in self.w]
        self.shapes = [l["dg"].shape for l in self.levels]

    def smooth(self, l, x, b):
        lv = self.levels[l]
        r = b if x is None else b - spmv(lv, x)
        d = line_solve(self.f[l], r)
        return (0.0 if x is None else x) + self.dtype(self.omega) * d

    def restrict(self, l, r):
        ft = 2 if self.shapes[l][1] > 1 else 1
        fp = 2 if self.shapes[l][0] > 1 else 1
        return _pair_sum(_pair_sum(self.w[l] * r, 1, ft), 0, fp)

    def prolong(self, l, xc):
        npf, ntf, _ = self.shapes[l]
        ft, fp = (2 if ntf > 1 else 1), (2 if npf > 1 else 1)
        return self.w[l] * _up(_up(xc, 1, ft, ntf), 0, fp, npf)

    def vcycle(self, b, l=0):
        """The cycle from level l on b."""
        if l == len(self.levels) - 1:
            return radial_solve(self.levels[l], b).astype(self.dtype)
        x = self.smooth(l, None, b)
        bc = self.restrict(l, b - spmv(self.levels[l], x))
        xc = self.kstep(l + 1, bc) if (l + 1) in self.klevels else self.vcycle(bc, l + 1)
        x = x + self.prolong(l, xc)
        return self.smooth(l, x, b)

    def kstep(self, l, b):
        """Two flexible-CG steps on level l, each preconditioned by the cycle from l."""
        lv = self.levels[l]
        dot = lambda u, v: float(np.sum(u.astype(np.float64) * v.astype(np.float64)))
        r = b.copy()
        z = self.vcycle(r, l)
        p = z
        q = spmv(lv, p)
        pq = dot(p, q)
        a = self.dtype(dot(p, r) / pq)
        x = a * p
        r = r - a * q
        z = self.vcycle(r, l)
        beta = self.dtype(-dot(z, q) / pq)
        p = z + beta * p
        q = spmv(lv, p)
        pq = dot(p, q)
        a = self.dtype(dot(p, r) / pq)
        return x + a * p

    def apply(self, r):
        """z = M_mg r for a flat residual (r fastest)."""
        sh = self.shapes[0]
        z = self.vcycle(np.asarray(r).astype(self.dtype).reshape(sh))
        return z.astype(np.float64).ravel()
