"""Pins of the network oracle (oracle/oracle_nn.c): conv taps against shifted copies,
adjoint (dot-product) identities for every backward routine, pooling/upsampling
invariants, a finite-difference check of the whole U-Net loss gradient, and the Adam
update against its closed form for a constant gradient."""
import numpy as np
import pytest

from oracle import NN

SHAPE = (6, 4, 4)
N = 6 * 4 * 4


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def _shifted(x, C, di, dj, dk):
    """x[i+di, j+dj, (k+dk) mod np] with zeros outside in r and theta (numpy roll + mask)."""
    nr, nt, npp = SHAPE
    a = x.reshape(npp, nt, nr, C)
    out = np.zeros_like(a)
    for k in range(npp):
        for j in range(nt):
            for i in range(nr):
                ii, jj, kk = i + di, j + dj, (k + dk) % npp
                if 0 <= ii < nr and 0 <= jj < nt:
                    out[k, j, i] = a[kk, jj, ii]
    return out.ravel()


@pytest.mark.parametrize("tap", [0, 4, 13, 14, 16, 22, 26])
def test_single_tap_kernel_is_a_shift(tap):
    cin, cout = 3, 3
    x = _rng(tap).standard_normal(N * cin)
    w = np.zeros((27, cout, cin))
    w[tap] = np.eye(3)
    y = NN.conv_fwd(SHAPE, x, cin, w, None, cout, relu=False)
    di, dj, dk = tap % 3 - 1, (tap // 3) % 3 - 1, tap // 9 - 1
    assert np.array_equal(y, _shifted(x, cin, di, dj, dk))


def test_bias_and_relu():
    x = np.zeros(N * 2)
    w = np.zeros((27, 2, 2))
    y = NN.conv_fwd(SHAPE, x, 2, w, np.array([1.5, -2.0]), 2, relu=True).reshape(N, 2)
    assert np.all(y[:, 0] == 1.5) and np.all(y[:, 1] == 0.0)


def test_backward_data_is_the_adjoint():
    r = _rng(1)
    cin, cout = 5, 3
    x = r.standard_normal(N * cin)
    dy = r.standard_normal(N * cout)
    w = r.standard_normal(27 * cout * cin)
    lhs = np.dot(NN.conv_fwd(SHAPE, x, cin, w, None, cout, False), dy)
    rhs = np.dot(x, NN.conv_bwd_data(SHAPE, dy, cout, w, cin))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_backward_weight_is_the_adjoint():
    r = _rng(2)
    cin, cout = 4, 2
    x = r.standard_normal(N * cin)
    dy = r.standard_normal(N * cout)
    w = r.standard_normal(27 * cout * cin)
    b = r.standard_normal(cout)
    dw, db = NN.conv_bwd_weight(SHAPE, x, cin, dy, cout)
    lhs = np.dot(NN.conv_fwd(SHAPE, x, cin, w, b, cout, False), dy)
    rhs = np.dot(dw, w) + np.dot(db, b)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_pool_and_up_are_adjoint_up_to_eight():
    r = _rng(3)
    C = 3
    xf = r.standard_normal(N * C)
    xc = r.standard_normal(N // 8 * C)
    # <pool(x), y> = <x, up(y)> / 8
    assert abs(np.dot(NN.pool(SHAPE, xf, C), xc) - np.dot(xf, NN.up(SHAPE, xc, C)) / 8) < 1e-12
    const = np.full(N * C, 2.5)
    assert np.allclose(NN.pool(SHAPE, const, C), 2.5)
    assert np.allclose(NN.up(SHAPE, np.full(N // 8 * C, -1.0), C), -1.0)


def _random_params(seed, scale=0.3):
    r = _rng(seed)
    p = np.empty(NN.param_count())
    for l, (taps, cout, cin) in enumerate(NN.layer_shapes()):
        o = NN.param_offset(l)
        nw = taps * cout * cin
        p[o:o + nw] = r.standard_normal(nw) * scale * np.sqrt(2.0 / (taps * cin))
        p[o + nw:o + nw + cout] = r.standard_normal(cout) * 0.1
    return p


def test_unet_gradient_matches_finite_differences():
    shape = (8, 4, 4)
    n = 8 * 4 * 4
    r = _rng(4)
    params = _random_params(5)
    X = np.zeros((n, 16))
    X[:, :4] = r.standard_normal((n, 4))
    e = r.standard_normal(n)
    L, grad, _ = NN.loss_grad(shape, params, X, e)
    picks = []
    for l, (taps, cout, cin) in enumerate(NN.layer_shapes()):
        o = NN.param_offset(l)
        nw = taps * cout * cin
        picks += [o + int(r.integers(nw)), o + nw + int(r.integers(cout))]
    for idx in picks:
        h = 1e-6 * max(1.0, abs(params[idx]))
        pp, pm = params.copy(), params.copy()
        pp[idx] += h
        pm[idx] -= h
        fd = (NN.loss_grad(shape, pp, X, e)[0] - NN.loss_grad(shape, pm, X, e)[0]) / (2 * h)
        # central differences carry a rounding error of ~eps * L / h ~ 1e-10 absolute;
        # a wrong or missing backward term is off by O(1) relative
        assert abs(fd - grad[idx]) <= 1e-5 * abs(grad[idx]) + 2e-9 * max(1.0, L), (idx, fd, grad[idx])


def test_loss_is_relative_l2():
    z = np.array([1.0, 2.0, 3.0])
    e = np.array([1.0, 1.0, 1.0])
    assert NN.loss_grad is not None
    from oracle import lib, _p
    gz = np.empty(3)
    L = lib().ognn_loss(3, _p(z), _p(e), _p(gz))
    assert abs(L - 5.0 / 3.0) < 1e-15
    assert np.allclose(gz, 2 * (z - e) / 3.0)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g, the bias-corrected moments are exactly g and g^2, so
    every step moves the parameter by lr * g / (|g| + eps)."""
    p0 = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m = np.zeros(3); v = np.zeros(3)
    p = p0.copy()
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    for t in range(1, 11):
        p, m, v = NN.adam(p, g, m, v, lr, b1, b2, eps, t)
    ref = p0 - 10 * lr * g / (np.abs(g) + eps)
    assert np.max(np.abs(p - ref)) < 1e-12


def _scaled_operator_sparse(shape, ahat):
    """The scaled operator as a scipy sparse matrix (unit diagonal, symmetric outward
    couplings, periodic in phi), built independently of the oracle's stencil loop."""
    import scipy.sparse as sp
    nr, nt, npp = shape
    n = nr * nt * npp
    a = np.asarray(ahat).reshape(3, npp, nt, nr)
    idx = np.arange(n).reshape(npp, nt, nr)
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [np.ones(n)]
    pairs = [(idx[:, :, :-1], idx[:, :, 1:], a[0][:, :, :-1]),
             (idx[:, :-1, :], idx[:, 1:, :], a[1][:, :-1, :])]
    if npp > 1:
        pairs.append((idx, np.roll(idx, -1, axis=0), a[2]))
    for i0, i1, v in pairs:
        rows += [i0.ravel(), i1.ravel()]
        cols += [i1.ravel(), i0.ravel()]
        vals += [v.ravel(), v.ravel()]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def test_residual_loss_value_and_gradient():
    shape = (8, 4, 4)
    n = 8 * 4 * 4
    r = _rng(6)
    params = _random_params(7)
    X = np.zeros((n, 16))
    X[:, :4] = r.standard_normal((n, 4))
    rr = r.standard_normal(n)
    ahat = -0.15 * r.random(3 * n)
    ahat.reshape(3, 4, 4, 8)[0][:, :, -1] = 0.0  # no coupling beyond the outer radial face
    ahat.reshape(3, 4, 4, 8)[1][:, -1, :] = 0.0  # nor beyond the last polar face
    L, grad, z = NN.loss_grad_resid(shape, params, X, rr, ahat)
    A = _scaled_operator_sparse(shape, ahat)
    q = A @ z
    assert abs(L - np.sum((q - rr) ** 2) / np.sum(rr ** 2)) <= 1e-12 * L
    picks = []
    for l, (taps, cout, cin) in enumerate(NN.layer_shapes()):
        o = NN.param_offset(l)
        nw = taps * cout * cin
        picks += [o + int(r.integers(nw)), o + nw + int(r.integers(cout))]
    for idx in picks:
        h = 1e-6 * max(1.0, abs(params[idx]))
        pp, pm = params.copy(), params.copy()
        pp[idx] += h
        pm[idx] -= h
        fd = (NN.loss_grad_resid(shape, pp, X, rr, ahat)[0] - NN.loss_grad_resid(shape, pm, X, rr, ahat)[0]) / (2 * h)
        assert abs(fd - grad[idx]) <= 1e-5 * abs(grad[idx]) + 2e-9 * max(1.0, L), (idx, fd, grad[idx])


def _bf16_numpy(x):
    """Round to bfloat16 (ties to even) via the float32 bit pattern, in numpy."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def test_bf16_rounding_is_round_to_nearest_even():
    """The oracle's bf16 rounding against a numpy bit-level round-to-nearest-even on
    ties, near-ties, subnormals, both signs and the overflow to infinity."""
    ulp = 2.0 ** -7
    xs = [1.0, 1.0 + ulp / 2, 1.0 + 1.5 * ulp, 1.0 + ulp / 2 + 2 ** -20, -(3.0 + ulp), 1e-39, -2.5e-40,
          3.3895e38, 3.4e38, 0.0]
    xs += list(_rng(5).standard_normal(2000) * 10.0 ** _rng(6).uniform(-30, 30, 2000))
    for x in xs:
        assert NN.bf16_round(x) == _bf16_numpy(np.float32(x)) or (np.isinf(NN.bf16_round(x)) and
                                                                   np.isinf(_bf16_numpy(np.float32(x))))
    assert NN.bf16_round(1.0 + ulp / 2) == 1.0 and NN.bf16_round(1.0 + 1.5 * ulp) == 1.0 + 2 * ulp
    assert np.isinf(NN.bf16_round(3.4e38))


def test_bf16_forward_is_the_layer_chain_with_rounded_activations():
    """The bf16-activation forward equals the composition of the oracle's own layers
    with every stored activation rounded (numpy rounding), exactly; it equals the fp64
    forward when every activation is already bf16-exact (small integers through
    single-tap integer weights); and it stays within bf16 rounding of the fp64 forward."""
    shape = (8, 8, 4)
    n = 8 * 8 * 4
    g = _rng(31)
    p = _random_params(31)
    X = _bf16_numpy(g.standard_normal(n * 16))
    z = NN.forward_bf16(shape, p, X)
    L = NN.layer_shapes()
    W = lambda l: p[NN.param_offset(l):NN.param_offset(l) + L[l][0] * L[l][1] * L[l][2]]
    B = lambda l: p[NN.param_offset(l) + L[l][0] * L[l][1] * L[l][2]:NN.param_offset(l + 1)]
    s1, s2, s3 = shape, tuple(d // 2 for d in shape), tuple(d // 4 for d in shape)
    q = _bf16_numpy
    a0 = q(NN.conv_fwd(s1, X, 16, W(0), B(0), 16, True))
    a1 = q(NN.conv_fwd(s1, a0, 16, W(1), B(1), 16, True))
    p1 = q(NN.pool(s1, a1, 16))
    a2 = q(NN.conv_fwd(s2, p1, 16, W(2), B(2), 32, True))
    a3 = q(NN.conv_fwd(s2, a2, 32, W(3), B(3), 32, True))
    p2 = q(NN.pool(s2, a3, 32))
    a4 = q(NN.conv_fwd(s3, p2, 32, W(4), B(4), 64, True))
    a5 = q(NN.conv_fwd(s3, a4, 64, W(5), B(5), 64, True))
    c6 = np.concatenate([NN.up(s2, a5, 64).reshape(-1, 64), a3.reshape(-1, 32)], axis=1).ravel()
    a6 = q(NN.conv_fwd(s2, c6, 96, W(6), B(6), 32, True))
    a7 = q(NN.conv_fwd(s2, a6, 32, W(7), B(7), 32, True))
    c8 = np.concatenate([NN.up(s1, a7, 32).reshape(-1, 32), a1.reshape(-1, 16)], axis=1).ravel()
    a8 = q(NN.conv_fwd(s1, c8, 48, W(8), B(8), 16, True))
    a9 = q(NN.conv_fwd(s1, a8, 16, W(9), B(9), 16, True))
    ref = a9.reshape(n, 16) @ W(10) + B(10)[0]
    assert np.max(np.abs(z - ref)) <= 1e-14 * np.max(np.abs(ref))
    _, _, z64 = NN.loss_grad(shape, p, X, np.ones(n))
    assert np.linalg.norm(z - z64) <= 0.05 * np.linalg.norm(z64)
    # integer-valued activations: channel 0 through the fine level only
    pi = np.zeros(NN.param_count())
    for l, ci in ((0, 0), (1, 0), (8, 32), (9, 0)):
        taps, cout, cin = L[l]
        pi[NN.param_offset(l) + (13 * cout + 0) * cin + ci] = 2.0
    pi[NN.param_offset(10)] = 1.0
    Xi = np.zeros((n, 16))
    Xi[:, 0] = g.integers(-8, 9, n)
    zi = NN.forward_bf16(shape, pi, Xi.ravel())
    _, _, zi64 = NN.loss_grad(shape, pi, Xi.ravel(), np.ones(n))
    assert np.array_equal(zi, zi64) and np.array_equal(zi, 16.0 * np.maximum(Xi[:, 0], 0))
