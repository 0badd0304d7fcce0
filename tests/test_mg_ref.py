"""Pins of the test-side multigrid reference (tests/mg_ref.py) against computations that
share none of its array arithmetic: explicit sparse products P^T A P, dense solves of
the phi-line matrices, the symmetry and definiteness a CG preconditioner needs, and the
iteration count of CG with it on a system the oracle assembled."""
import numpy as np
import pytest
import scipy.sparse as sp

import mg_ref


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def _random_operator(shape, seed):
    """A^-like couplings (negative, zero on the boundary faces, periodic phi) and s > 0."""
    nr, nt, nph = shape
    r = _rng(seed)
    a = -r.uniform(0.02, 0.3, (3, nph, nt, nr))
    a[0, :, :, -1] = 0.0
    a[1, :, -1, :] = 0.0
    if nph == 1:
        a[2] = 0.0
    s = np.exp(r.uniform(-3, 3, (nph, nt, nr)))
    return a.ravel(), s.ravel()


def _csr(lv):
    """The level's operator as a sparse matrix, entry by entry from the 7-point arrays."""
    dg, ar, at, ap = lv["dg"], lv["ar"], lv["at"], lv["ap"]
    nph, nt, nr = dg.shape
    idx = lambda i, j, k: i + nr * (j + nt * k)
    rows, cols, vals = [], [], []
    for k in range(nph):
        for j in range(nt):
            for i in range(nr):
                c = idx(i, j, k)
                rows.append(c); cols.append(c); vals.append(dg[k, j, i])
                nb = []
                if i + 1 < nr:
                    nb.append((idx(i + 1, j, k), ar[k, j, i]))
                if j + 1 < nt:
                    nb.append((idx(i, j + 1, k), at[k, j, i]))
                if nph > 1:
                    nb.append((idx(i, j, (k + 1) % nph), ap[k, j, i]))
                for g, v in nb:
                    rows += [c, g]; cols += [g, c]; vals += [v, v]
    n = nr * nt * nph
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def _prolongation(shape, B):
    """P[f, C] = B_f / ||B on C||: aggregates of the theta and phi pairs (radius kept)."""
    nr, nt, nph = shape
    ft, fp = (2 if nt > 1 else 1), (2 if nph > 1 else 1)
    ntc, npc = (nt + ft - 1) // ft, (nph + fp - 1) // fp
    B = B.reshape(nph, nt, nr)
    rows, cols, vals = [], [], []
    for k in range(nph):
        for j in range(nt):
            for i in range(nr):
                rows.append(i + nr * (j + nt * k))
                cols.append(i + nr * (j // ft + ntc * (k // fp)))
                vals.append(B[k, j, i])
    P = sp.csr_matrix((vals, (rows, cols)), shape=(nr * nt * nph, nr * ntc * npc))
    norms = np.sqrt(np.asarray(P.multiply(P).sum(axis=0))).ravel()
    return (P @ sp.diags(1.0 / norms)).tocsr(), (nr, ntc, npc), norms


SHAPES = [(6, 4, 8), (5, 7, 5), (4, 6, 3), (3, 5, 2), (7, 6, 1), (4, 1, 6), (3, 1, 1)]


@pytest.mark.parametrize("shape", SHAPES)
def test_levels_are_galerkin_products(shape):
    """Every level equals P^T A P of the level above, built here as sparse matrices."""
    a, s = _random_operator(shape, 3)
    H = mg_ref.Hierarchy(shape, a, s)
    A = _csr(H.levels[0])
    B = 1.0 / s
    sh = shape
    for l in range(len(H.levels) - 1):
        P, sh, B = _prolongation(sh, B)
        Ac = (P.T @ A @ P).toarray()
        got = _csr(H.levels[l + 1]).toarray()
        assert got.shape == Ac.shape
        assert np.allclose(got, Ac, rtol=1e-12, atol=1e-12 * np.abs(Ac).max()), (shape, l)
        w = H.w[l].ravel()
        assert np.allclose(w, P.toarray().sum(axis=1))
        A = sp.csr_matrix(Ac)
    assert H.shapes[-1][:2] == (1, 1)


@pytest.mark.parametrize("shape", SHAPES)
def test_spmv_matches_the_sparse_matrix(shape):
    a, s = _random_operator(shape, 5)
    H = mg_ref.Hierarchy(shape, a, s)
    x = _rng(6).standard_normal(shape[::-1])
    for lv in H.levels:
        xl = x[:lv["dg"].shape[0], :lv["dg"].shape[1], :]
        assert np.allclose(mg_ref.spmv(lv, xl).ravel(), _csr(lv) @ xl.ravel(), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("nph", [1, 2, 3, 4, 9])
def test_line_solve_is_the_inverse_of_the_phi_line_matrix(nph):
    """The Sherman-Morrison line solve against a dense solve of each (r, theta) line's
    diagonal-plus-phi block (periodic; two couplings between the cells of a 2-line)."""
    shape = (3, 2, nph)
    a, s = _random_operator(shape, 7)
    H = mg_ref.Hierarchy(shape, a, s)
    lv = H.levels[0]
    f = mg_ref.line_factors(lv)
    rhs = _rng(8).standard_normal((nph, 2, 3))
    x = mg_ref.line_solve(f, rhs)
    for j in range(2):
        for i in range(3):
            M = np.diag(lv["dg"][:, j, i].copy())
            for k in range(nph if nph > 1 else 0):
                kn = (k + 1) % nph
                M[k, kn] += lv["ap"][k, j, i]
                M[kn, k] += lv["ap"][k, j, i]
            assert np.allclose(x[:, j, i], np.linalg.solve(M, rhs[:, j, i]), rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("shape", [(6, 4, 8), (5, 7, 5), (7, 6, 1)])
def test_vcycle_is_symmetric_positive_definite(shape):
    """Without K-cycle steps the cycle is a fixed linear operator, and CG needs it
    symmetric positive definite: u.M v = v.M u, u.M u > 0."""
    a, s = _random_operator(shape, 9)
    H = mg_ref.Hierarchy(shape, a, s, klevels=())
    r = _rng(10)
    n = int(np.prod(shape))
    for _ in range(4):
        u, v = r.standard_normal(n), r.standard_normal(n)
        Mu, Mv = H.apply(u), H.apply(v)
        assert abs(u @ Mv - v @ Mu) <= 1e-12 * np.linalg.norm(u) * np.linalg.norm(Mv)
        assert u @ Mu > 0


@pytest.mark.parametrize("shape", [(6, 16, 8), (5, 9, 12)])
def test_kcycle_step_is_the_galerkin_projection_on_its_two_directions(shape):
    """Two CG steps with a fixed SPD preconditioner M from zero give the A-orthogonal
    projection of A^-1 b on span{z1, z2} (z1 = M b, z2 = M (b - a1 A z1)): checked against
    the 2 x 2 Galerkin system solved densely, on a level whose own cycle is linear (the
    K level's preconditioner is the V-cycle below it)."""
    a, s = _random_operator(shape, 13)
    H = mg_ref.Hierarchy(shape, a, s, klevels=(1,))
    assert H.klevels == (1,)
    lv = H.levels[1]
    A = _csr(lv).toarray()
    b = _rng(14).standard_normal(lv["dg"].shape)
    x = H.kstep(1, b)
    M = lambda v: H.vcycle(v, 1)
    z1 = M(b)
    a1 = (z1.ravel() @ b.ravel()) / (z1.ravel() @ A @ z1.ravel())
    z2 = M(b - a1 * (A @ z1.ravel()).reshape(b.shape))
    V = np.stack([z1.ravel(), z2.ravel()], axis=1)
    c = np.linalg.solve(V.T @ A @ V, V.T @ b.ravel())
    assert np.allclose(x.ravel(), V @ c, rtol=1e-10, atol=1e-12 * np.abs(V @ c).max())


def test_vcycle_on_one_radial_line_is_the_exact_solve():
    shape = (9, 1, 1)
    a, s = _random_operator(shape, 11)
    H = mg_ref.Hierarchy(shape, a, s)
    A = _csr(H.levels[0]).toarray()
    b = _rng(12).standard_normal(9)
    assert np.allclose(A @ H.apply(b), b, rtol=1e-12, atol=1e-12)


def _pcg(A, b, M, tol=1e-8, maxit=3000):
    x = np.zeros_like(b); r = b.copy(); z = M(r); p = z.copy(); rz = r @ z; bn = np.linalg.norm(b)
    for it in range(1, maxit + 1):
        q = A @ p
        al = rz / (p @ q)
        x += al * p; r -= al * q
        if np.linalg.norm(r) <= tol * bn:
            return it, x
        z = M(r); rz2 = r @ z; p = z + rz2 / rz * p; rz = rz2
    return maxit, x


def _fcg(A, b, M, tol=1e-8, maxit=3000):
    """Flexible CG (beta = -(z.q_old)/(p_old.q_old)), as the solver runs it."""
    x = np.zeros_like(b); r = b.copy(); bn = np.linalg.norm(b); p = q = pq = None
    for it in range(1, maxit + 1):
        z = M(r)
        p = z.copy() if p is None else z - (z @ q) / pq * p
        q = A @ p
        pq = p @ q
        al = (p @ r) / pq
        x += al * p; r -= al * q
        if np.linalg.norm(r) <= tol * bn:
            return it, x
    return maxit, x


def test_cg_with_the_vcycle_on_an_oracle_system():
    """On the system the oracle assembles for a clumpy 32 x 16 x 32 grid, CG with one
    V-cycle per iteration meets 1e-8 in at most 25 iterations (Jacobi CG takes about ten
    times as many), in float64 and with the cycle in float32; flexible CG with the
    K-cycle in at most 12."""
    import oracle
    from paper_1001_3301_amd import synth as sy
    shape = (32, 16, 32)
    wl = sy.make_workload("mg-pin", *shape, 16, 100.0, clump_seed=3000)
    P = oracle.Problem.from_workload(wl)
    rh = wl.rho.ravel()
    To = np.full(P.n, wl.T_bc)
    _, So, _ = P.raytrace(rh, To, want_faces=False)
    To = P.newton(np.full(P.n, sy.A_RAD * wl.T_bc ** 4), So, To)
    qo, So, _ = P.raytrace(rh, To, want_faces=False)
    out = P.assemble(rh, To, P.energy(To, So), qo)
    H = mg_ref.Hierarchy(shape, out["ahat"], out["s"], klevels=())
    A = _csr(H.levels[0])
    b = out["bhat"]
    it_cg, _ = _pcg(A, b, lambda r: r)
    for dt in (np.float64, np.float32):
        Hd = mg_ref.Hierarchy(shape, out["ahat"], out["s"], dtype=dt, klevels=())
        it, x = _pcg(A, b, Hd.apply)
        assert it <= 25, (dt, it, it_cg)
        assert P.relres(out["ahat"], b, x) <= 1e-8
    assert it_cg >= 5 * it
    Hk = mg_ref.Hierarchy(shape, out["ahat"], out["s"], dtype=np.float32)
    assert Hk.klevels == (1, 2, 3)
    itk, x = _fcg(A, b, Hk.apply)
    assert itk <= 12 and itk < it, (itk, it)
    assert P.relres(out["ahat"], b, x) <= 1e-8
