"""GPU parity of the learned preconditioner (BF16 MFMA kernels) with the float64 oracle.

Layer level: the HIP convolution forward, data gradient and weight gradient against
oracle/oracle_nn.c on the same BF16-rounded operands (inputs, weights, and the
gradients fed in), FP32 accumulation vs FP64: <= 1e-5 of the output's magnitude.
Network level: the whole forward / gradient (which round activations to BF16 between
layers) against the FP64 oracle with loose bounds; training lowers the loss; the
learned solve meets the float64 tolerance and falls back when the network misbehaves.
"""
import numpy as np
import pytest

from oracle import NN
from paper_1001_3301_amd import synth as sy

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def bf16_bits(x):
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def bits_to_f64(b):
    return (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def dev_bf16(bits):
    return torch.from_numpy(bits.view(np.int16).copy()).view(torch.bfloat16).cuda()


def dev_f32(x):
    return torch.tensor(np.ascontiguousarray(x, dtype=np.float32).ravel(), device="cuda")


def up_np(shape, xc, C):
    return NN.up(shape, xc, C)


def concat(a, ca, b, cb, n):
    if cb == 0:
        return a
    return np.concatenate([a.reshape(n, ca), b.reshape(n, cb)], axis=1).ravel()


CONV_CASES = [
    # shape (fine), c1, up1, c2, cout
    ((10, 6, 4), 16, 0, 0, 16),
    ((10, 6, 4), 16, 0, 0, 32),
    ((8, 4, 4), 32, 0, 0, 64),
    ((6, 4, 6), 64, 0, 0, 64),
    ((8, 8, 4), 64, 1, 32, 32),   # decoder: up(coarse 64) + skip 32
    ((12, 8, 4), 32, 1, 16, 16),  # decoder: up(coarse 32) + skip 16
]


# Tiles are 32 radial cells x TJ x TK (TJ, TK in {4, 2}); 72 x 10 x 6 gives two full
# radial tiles and a partial one, and partial theta and phi tiles, for every
# (output tiles, TJ, TK) instantiation of the forward and data-gradient kernels
# (cout 16/32 -> <1|2,4,4>, 48/64 -> <3|4,4,2>; data gradient of 96 channels -> <6,2,2>)
# and every weight-gradient width.
FULL_TILE_CASES = [
    ((72, 10, 6), 16, 0, 0, 16),
    ((72, 10, 6), 16, 0, 0, 32),
    ((72, 10, 6), 16, 0, 0, 48),
    ((72, 10, 6), 32, 0, 0, 64),
    ((72, 10, 6), 64, 0, 0, 64),
    ((72, 10, 6), 64, 1, 32, 32),
    ((72, 10, 6), 32, 1, 16, 16),
]
CONV_CASES_ALL = CONV_CASES + FULL_TILE_CASES
# The 16 -> 16 forward convolutions walk phi in chunks of 32 planes with 32 x 8 cell
# columns: 70 phi planes give two full chunks and a partial one (whose halo wraps to
# plane 0), 18 theta rows two full and a partial theta tile; also with the upsampled input.
# The fine decoder layer (up(32) + skip 16 -> 16) walks 32 x 16 columns over the same
# chunks with the coarse planes in its ring: 40 x 36 x 68 crosses r tiles (32 + 8), theta
# tiles (16 + 16 + 4) and phi chunks (32 + 32 + 4); 44 x 20 x 38 has odd coarse
# dimensions (22 x 10 x 19) and a phi chunk of 6 planes.
SLIDE_CASES = [
    ((72, 18, 70), 16, 0, 0, 16),
    ((40, 12, 36), 16, 1, 0, 16),
    ((40, 36, 68), 32, 1, 16, 16),
    ((44, 20, 38), 32, 1, 16, 16),
]


def _conv_inputs(case, seed):
    shape, c1, up1, c2, cout = case
    nr, nt, npp = shape
    n = nr * nt * npp
    n1 = n // 8 if up1 else n
    r = _rng(seed)
    x1 = bf16_bits(r.standard_normal(n1 * c1))
    x2 = bf16_bits(r.standard_normal(n * c2)) if c2 else None
    cin = c1 + c2
    w = bf16_bits(r.standard_normal(27 * cout * cin) * 0.2)
    b = r.standard_normal(cout).astype(np.float32)
    x1f = bits_to_f64(x1)
    xin = up_np(shape, x1f, c1) if up1 else x1f
    xcat = concat(xin, c1, None if x2 is None else bits_to_f64(x2), c2, n)
    return n, x1, x2, w, b, xcat, cin


@pytest.mark.parametrize("case", CONV_CASES_ALL + SLIDE_CASES, ids=[str(c) for c in CONV_CASES_ALL + SLIDE_CASES])
def test_conv_forward_parity(case):
    from paper_1001_3301_amd import rt
    shape, c1, up1, c2, cout = case
    n, x1, x2, w, b, xcat, cin = _conv_inputs(case, 1)
    yf = torch.empty(n * cout, dtype=torch.float32, device="cuda")
    rt.nn_conv_fwd(shape, dev_bf16(x1), c1, up1, None if x2 is None else dev_bf16(x2), c2, dev_bf16(w),
                   dev_f32(b), cout, True, None, yf)
    ref = NN.conv_fwd(shape, xcat, cin, bits_to_f64(w), b.astype(np.float64), cout, True)
    got = yf.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref))


def _pool_bits_host(shape, ybits):
    """2x2x2 average of bf16 values (bits), summed in float32 in the order r, theta, phi and
    rounded to bf16 (round to nearest even): the arithmetic of the network's pooling."""
    nr, nt, npp = shape
    yv = bits_to_f64(ybits).astype(np.float32).reshape(npp, nt, nr, 16)
    s = np.zeros((npp // 2, nt // 2, nr // 2, 16), dtype=np.float32)
    for q in range(8):
        dr, dt, dp = q & 1, (q >> 1) & 1, q >> 2
        s = (s + yv[dp::2, dt::2, dr::2]).astype(np.float32)
    return bf16_bits((s * np.float32(0.125)).astype(np.float32)).reshape(-1)


@pytest.mark.parametrize("shape", [(72, 18, 70), (40, 12, 36), (8, 4, 4)], ids=str)
def test_conv_with_pooling_in_one_pass(shape):
    """rt_nn_conv3d_fwd_pool: y the same bits as rt_nn_conv3d_fwd (16 -> 16, ReLU), its
    pool the same bits as the 2x2x2 average of y in float32 (r, theta, phi order), and both
    against the oracle (conv and pool of the same bf16 operands in float64).  72 x 18 x 70
    crosses r and theta tiles and phi chunks (with a partial one)."""
    from paper_1001_3301_amd import rt
    case = (shape, 16, 0, 0, 16)
    n, x1, x2, w, b, xcat, cin = _conv_inputs(case, 11)
    nc = n // 8
    y = torch.empty(n * 16, dtype=torch.bfloat16, device="cuda")
    yp = torch.empty(nc * 16, dtype=torch.bfloat16, device="cuda")
    y2 = torch.empty(n * 16, dtype=torch.bfloat16, device="cuda")
    rt.nn_conv_fwd_pool(shape, dev_bf16(x1), dev_bf16(w), dev_f32(b), y, yp)
    rt.nn_conv_fwd(shape, dev_bf16(x1), 16, 0, None, 0, dev_bf16(w), dev_f32(b), 16, True, y2, None)
    yb = y.view(torch.int16).cpu().numpy().view(np.uint16)
    assert np.array_equal(yb, y2.view(torch.int16).cpu().numpy().view(np.uint16))
    pb = yp.view(torch.int16).cpu().numpy().view(np.uint16)
    assert np.array_equal(pb, _pool_bits_host(shape, yb))
    ref = NN.conv_fwd(shape, xcat, 16, bits_to_f64(w), b.astype(np.float64), 16, True)
    refp = NN.pool(shape, ref, 16)
    assert np.max(np.abs(bits_to_f64(yb) - ref)) <= 2.0 ** -8 * np.max(np.abs(ref))
    assert np.max(np.abs(bits_to_f64(pb) - refp)) <= 2.0 ** -7 * np.max(np.abs(refp))


@pytest.mark.parametrize("case", CONV_CASES_ALL, ids=[str(c) for c in CONV_CASES_ALL])
def test_conv_backward_parity(case):
    from paper_1001_3301_amd import rt
    shape, c1, up1, c2, cout = case
    n, x1, x2, w, b, xcat, cin = _conv_inputs(case, 2)
    r = _rng(3)
    dy = bits_to_f64(bf16_bits(r.standard_normal(n * cout)))  # already bf16-representable
    yr = bf16_bits(r.standard_normal(n * cout))                # ReLU output mask source
    dym = dy * (bits_to_f64(yr) > 0)
    # transposed weights for the data gradient
    wt = bf16_bits(bits_to_f64(w).reshape(27, cout, cin).transpose(0, 2, 1).ravel())
    d1 = torch.empty(n * c1, dtype=torch.float32, device="cuda")
    d2 = torch.empty(n * c2, dtype=torch.float32, device="cuda") if c2 else None
    rt.nn_conv_bwd_data(shape, dev_f32(dy), dev_bf16(yr), cout, dev_bf16(wt), c1, d1, c2, d2)
    ref = NN.conv_bwd_data(shape, dym, cout, bits_to_f64(w), cin).reshape(n, cin)
    got = d1.cpu().numpy().reshape(n, c1)
    if c2:
        got = np.concatenate([got, d2.cpu().numpy().reshape(n, c2)], axis=1)
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref))
    dw = torch.empty(27 * cout * cin, dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    rt.nn_conv_bwd_weight(shape, dev_f32(dy), dev_bf16(yr), cout, dev_bf16(x1), c1, up1,
                          None if x2 is None else dev_bf16(x2), c2, dw, db)
    rdw, rdb = NN.conv_bwd_weight(shape, xcat, cin, dym, cout)
    assert np.max(np.abs(dw.cpu().numpy() - rdw)) <= 1e-5 * np.max(np.abs(rdw))
    assert np.max(np.abs(db.cpu().numpy() - rdb)) <= 1e-5 * np.max(np.abs(rdb))


def _ctx_for(shape, n_nu=8, tau=10.0, seed=4):
    from paper_1001_3301_amd import rt
    wl = sy.make_workload("unet-test", shape[0], shape[1], shape[2], n_nu, tau, clump_seed=seed)
    return wl, rt.Context.from_workload(wl)


def _net_input(n, seed):
    r = _rng(seed)
    X = np.zeros((n, 16), dtype=np.float32)
    X[:, 0] = r.standard_normal(n)
    X[:, 1:4] = r.uniform(-1, 1, (n, 3))
    return bf16_bits(X.ravel())


def test_network_forward_and_gradient_against_oracle():
    from paper_1001_3301_amd import rt
    shape = (16, 8, 8)
    n = 16 * 8 * 8
    wl, ctx = _ctx_for(shape)
    net = rt.Net(seed=7)
    p = net.get_params().astype(np.float64)
    # the oracle gets the weights the GPU computes with (bf16-rounded), biases in fp32
    pq = p.copy()
    for l, (taps, cout, cin) in enumerate(NN.layer_shapes()):
        o = NN.param_offset(l)
        nw = taps * cout * cin
        pq[o:o + nw] = bits_to_f64(bf16_bits(p[o:o + nw]))
    Xb = _net_input(n, 8)
    X64 = bits_to_f64(Xb).reshape(n, 16)
    e = _rng(9).standard_normal(n).astype(np.float32)
    z = torch.empty(n, dtype=torch.float32, device="cuda")
    net.forward(ctx, dev_bf16(Xb), z)
    L_ref, g_ref, z_ref = NN.loss_grad(shape, pq, X64, e.astype(np.float64))
    zg = z.cpu().numpy().astype(np.float64)
    # activations are rounded to bf16 after every layer on the GPU
    assert np.linalg.norm(zg - z_ref) <= 3e-2 * np.linalg.norm(z_ref)
    L = net.loss_grad(ctx, dev_bf16(Xb), dev_f32(e))
    assert abs(L - L_ref) <= 3e-2 * L_ref
    g = net.get_grads().astype(np.float64)
    for l, (taps, cout, cin) in enumerate(NN.layer_shapes()):
        o = NN.param_offset(l)
        sl = slice(o, o + taps * cout * cin + cout)
        a, b = g[sl], g_ref[sl]
        cos = np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300)
        assert cos > 0.99, (l, cos)
        assert np.linalg.norm(a - b) <= 0.1 * np.linalg.norm(b), l


def _bf16_weights(p):
    """The parameters as the GPU computes with them: bf16-rounded weights, fp32 biases."""
    pq = p.astype(np.float64).copy()
    for l, (taps, cout, cin) in enumerate(NN.layer_shapes()):
        o = NN.param_offset(l)
        nw = taps * cout * cin
        pq[o:o + nw] = bits_to_f64(bf16_bits(p[o:o + nw]))
    return pq


@pytest.mark.parametrize("seed", [7, 8])
def test_network_forward_against_bf16_oracle_on_a_multi_tile_grid(seed):
    """rt_net_forward at 64 x 32 x 32 (level-0 layers span two radial tiles, 8 x 8 theta-phi
    tiles; every level and the decoder's upsampled reads cross tiles) against the oracle's
    forward with the same bf16 storage of every activation, element by element.  The
    remaining difference is fp32 against fp64 accumulation, which moves an activation to
    the neighbouring bf16 value where it lies close to a rounding boundary (a sum of up to
    2592 products with cancellation carries fp32 errors of ~1e-5 of itself); such flips
    (one bf16 ulp, 2^-7) spread through the following layers' receptive fields: measured
    relative L2 3.4e-3 - 5.2e-3, median 3.5e-4 - 7.5e-4 of the largest output."""
    from paper_1001_3301_amd import rt
    shape = (64, 32, 32)
    n = 64 * 32 * 32
    wl, ctx = _ctx_for(shape)
    net = rt.Net(seed=seed)
    pq = _bf16_weights(net.get_params())
    Xb = _net_input(n, seed + 100)
    X64 = bits_to_f64(Xb)
    z = torch.empty(n, dtype=torch.float32, device="cuda")
    net.forward(ctx, dev_bf16(Xb), z)
    ref = NN.forward_bf16(shape, pq, X64)
    zg = z.cpu().numpy().astype(np.float64)
    d = np.abs(zg - ref) / np.max(np.abs(ref))
    rel2 = np.linalg.norm(zg - ref) / np.linalg.norm(ref)
    print(f"seed {seed}: rel L2 {rel2:.3e}, max {d.max():.3e}, p99 {np.quantile(d, 0.99):.3e}, "
          f"median {np.median(d):.3e}, exact cells {np.mean(d == 0):.3f}")
    assert rel2 <= 1e-2 and d.max() <= 3e-2
    assert np.median(d) <= 2e-3


def test_forward_with_fused_output_layer_equals_the_layer_by_layer_forward():
    """rt_net_forward runs the last convolution and the 1x1 output layer as one kernel
    (the hidden activation is not written); rt_net_loss_grad, which keeps that activation
    for its backward pass, runs them as two.  z agrees bit for bit.  On 72 x 36 x 68 the
    fine level spans full and partial r tiles, theta tiles and phi chunks."""
    from paper_1001_3301_amd import rt
    shape = (72, 36, 68)
    n = 72 * 36 * 68
    wl, ctx = _ctx_for(shape)
    net = rt.Net(seed=5)
    Xb = _net_input(n, 31)
    z1 = torch.empty(n, dtype=torch.float32, device="cuda")
    z2 = torch.empty(n, dtype=torch.float32, device="cuda")
    net.forward(ctx, dev_bf16(Xb), z1)
    net.loss_grad(ctx, dev_bf16(Xb), dev_f32(_rng(32).standard_normal(n)), z2)
    a, b = z1.cpu().numpy(), z2.cpu().numpy()
    assert np.all(np.isfinite(a)) and np.abs(a).max() > 0
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_adam_step_matches_formula():
    from paper_1001_3301_amd import rt
    shape = (8, 4, 4)
    n = 8 * 4 * 4
    wl, ctx = _ctx_for(shape)
    net = rt.Net(seed=3)
    p0 = net.get_params().astype(np.float64)
    Xb = _net_input(n, 1)
    e = _rng(2).standard_normal(n).astype(np.float32)
    net.loss_grad(ctx, dev_bf16(Xb), dev_f32(e))
    g = net.get_grads().astype(np.float64)
    net.adam(ctx, 1e-3)
    p1 = net.get_params().astype(np.float64)
    ref, _, _ = NN.adam(p0, g, np.zeros_like(p0), np.zeros_like(p0), 1e-3, 0.9, 0.999, 1e-8, 1)
    assert np.max(np.abs(p1 - ref)) <= 1e-6 * max(1.0, np.max(np.abs(p0)))


def _small_problem(shape=(32, 16, 16), tau=10.0, seed=5):
    """Context with an assembled system of a clumpy workload, and E^n on the device."""
    return _small_problem_sys(shape, tau, seed)[:6]


def _small_problem_sys(shape=(32, 16, 16), tau=10.0, seed=5):
    """_small_problem, plus the device view of the assembled system."""
    wl, ctx = _ctx_for(shape, n_nu=16, tau=tau, seed=seed)
    n = ctx.n
    rho = torch.tensor(wl.rho.ravel(), device="cuda")
    T = torch.full((n,), wl.T_bc, dtype=torch.float64, device="cuda")
    q = torch.empty(n, dtype=torch.float64, device="cuda"); S = torch.empty_like(q)
    ctx.raytrace(rho, T, q, S)
    ctx.temperature(torch.full((n,), sy.A_RAD * wl.T_bc ** 4, dtype=torch.float64, device="cuda"), S, T)
    ctx.raytrace(rho, T, q, S)
    En = torch.empty_like(q)
    ctx.energy(T, S, En)
    sysv = ctx.assemble(rho, T, En, q)
    return wl, ctx, rho, T, En, S, sysv


def test_training_lowers_the_loss_and_learned_solve_converges(tmp_path):
    from paper_1001_3301_amd import rt
    wl, ctx, rho, T, En, S = _small_problem()
    ds = rt.Dataset(ctx, 12)
    ds.add(En, [0, 5, 20, 60])
    assert len(ds) == 4
    net = rt.Net(seed=11)
    st = net.train(ctx, ds, epochs=25, lr=2e-3, seed=1)
    assert st["steps"] == 100
    assert st["loss_last_epoch"] < 0.7 * st["loss_first_epoch"], st
    # save / load round trip
    path = tmp_path / "net.bin"
    net.save(path)
    net2 = rt.Net(seed=99)
    net2.load(path)
    assert np.array_equal(net2.get_params(), net.get_params())
    # the learned solve meets the float64 tolerance and agrees with the float64 solve
    E_l = En.clone()
    rc, sl = ctx.solve(E_l, rt.solve_opts(rt.MODE_LEARNED, tol=1e-8, net=net))
    assert sl["relres"] <= 1e-8 and sl["precond_applies"] > 0
    E_f = En.clone()
    rc, sf = ctx.solve(E_f, rt.solve_opts(rt.MODE_FP64, tol=1e-10))
    Tl, Tf = T.clone(), T.clone()
    ctx.temperature(E_l, S, Tl)
    ctx.temperature(E_f, S, Tf)
    assert float(((Tl - Tf).abs() / Tf).max()) < 1e-3


@pytest.mark.parametrize("inner", [0, 1], ids=["fcg", "fgmres"])
def test_learned_solve_falls_back_when_the_network_blows_up(inner):
    from paper_1001_3301_amd import rt
    wl, ctx, rho, T, En, S = _small_problem(shape=(16, 8, 8))
    net = rt.Net(seed=2)
    p = net.get_params()
    net.set_params(np.full_like(p, 1e30))  # finite weights, overflowing activations
    E = En.clone()
    rc, st = ctx.solve(E, rt.solve_opts(rt.MODE_LEARNED, tol=1e-8, net=net, inner=inner))
    assert st["fallback"] == 1 and st["handover"] == 0 and st["relres"] <= 1e-8
    assert np.all(np.isfinite(E.cpu().numpy()))


def test_conv_blocks_serving_several_tiles_against_oracle():
    """The persistent grid holds at most 256 compute units x the blocks that fit on one
    (by LDS), so on the training and inference grids every block walks several tiles.
    64 x 64 x 128 has 1024 tiles of 32 x 4 x 4 cells, more than the grid: the forward
    decoder layer (coarse 32 channels upsampled + 16 skip -> 16, three input slices per
    tile) and the 16 -> 16 data gradient against the oracle, every output compared."""
    from paper_1001_3301_amd import rt
    case = ((64, 64, 128), 32, 1, 16, 16)
    shape, c1, up1, c2, cout = case
    n, x1, x2, w, b, xcat, cin = _conv_inputs(case, 21)
    yf = torch.empty(n * cout, dtype=torch.float32, device="cuda")
    rt.nn_conv_fwd(shape, dev_bf16(x1), c1, up1, dev_bf16(x2), c2, dev_bf16(w), dev_f32(b), cout, True, None, yf)
    ref = NN.conv_fwd(shape, xcat, cin, bits_to_f64(w), b.astype(np.float64), cout, True)
    got = yf.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref))
    shape, cout, cin = (64, 64, 128), 16, 16
    n = 64 * 64 * 128
    r = _rng(22)
    w = bf16_bits(r.standard_normal(27 * cout * cin) * 0.2)
    dy = bits_to_f64(bf16_bits(r.standard_normal(n * cout)))
    yr = bf16_bits(r.standard_normal(n * cout))
    dym = dy * (bits_to_f64(yr) > 0)
    wt = bf16_bits(bits_to_f64(w).reshape(27, cout, cin).transpose(0, 2, 1).ravel())
    d1 = torch.empty(n * cin, dtype=torch.float32, device="cuda")
    rt.nn_conv_bwd_data(shape, dev_f32(dy), dev_bf16(yr), cout, dev_bf16(wt), cin, d1, 0, None)
    ref = NN.conv_bwd_data(shape, dym, cout, bits_to_f64(w), cin)
    assert np.max(np.abs(d1.cpu().numpy() - ref)) <= 1e-5 * np.max(np.abs(ref))


@pytest.mark.parametrize("case", [((64, 64, 32), 16, 0, 0, 16), ((64, 64, 32), 32, 1, 16, 16)],
                         ids=["16-16", "up32+16-16"])
def test_weight_gradient_over_more_tiles_than_blocks(case):
    """The weight-gradient grid is capped at 256 blocks per input slice; 64 x 64 x 32
    has 1024 tiles of 32 x 2 x 2 cells, so each block accumulates four tiles before the
    fixed-order sum of the partials.  Every weight and bias against the oracle."""
    from paper_1001_3301_amd import rt
    shape, c1, up1, c2, cout = case
    n, x1, x2, w, b, xcat, cin = _conv_inputs(case, 23)
    r = _rng(24)
    dy = bits_to_f64(bf16_bits(r.standard_normal(n * cout)))
    yr = bf16_bits(r.standard_normal(n * cout))
    dym = dy * (bits_to_f64(yr) > 0)
    dw = torch.empty(27 * cout * cin, dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    rt.nn_conv_bwd_weight(shape, dev_f32(dy), dev_bf16(yr), cout, dev_bf16(x1), c1, up1,
                          None if x2 is None else dev_bf16(x2), c2, dw, db)
    rdw, rdb = NN.conv_bwd_weight(shape, xcat, cin, dym, cout)
    assert np.max(np.abs(dw.cpu().numpy() - rdw)) <= 1e-5 * np.max(np.abs(rdw))
    assert np.max(np.abs(db.cpu().numpy() - rdb)) <= 1e-5 * np.max(np.abs(rdb))


def _identity_path_params(gain, out_scale):
    """Parameters of a network that passes channel 0 of its input through the fine
    level only: z = out_scale * relu(gain * x0) (centre taps of layers 0, 1, 8, 9 and the
    output layer; every other weight and bias zero).  The gain sits in the decoder layer
    that reads the skip connection (layer 8), after the pooling into the coarse levels,
    whose fp32 sums of eight activations would otherwise overflow first; gain * x0
    overflows float32 (and so bf16) there where x0 > 3.4e38 / gain."""
    p = np.zeros(NN.param_count(), dtype=np.float32)
    centre = 13  # (dk, dj, di) = (0, 0, 0)
    for l, ci, g in ((0, 0, 1.0), (1, 0, 1.0), (8, 32, gain), (9, 0, 1.0)):
        taps, cout, cin = NN.layer_shapes()[l]
        p[NN.param_offset(l) + (centre * cout + 0) * cin + ci] = g
    p[NN.param_offset(10)] = out_scale
    return p


def test_learned_reduced_finish_recovers_from_a_network_that_overflows_on_its_second_application():
    """A network whose output is finite on the first residual and overflows on the
    second: the non-finite exit happens after the flexible CG wrote the network's output
    into the direction buffer that the reduced finish starts from.  The finish must
    restart from zero directions (p = r) and meet the tolerance; `fallback` reports the
    failed network.  The overflow threshold is set between the largest entries of the
    unit-RMS first and second residuals, computed on the host from the GPU's own
    assembled system with the identity-path network's first FCG step."""
    from paper_1001_3301_amd import rt
    wl, ctx, rho, T, En, S, sysv = _small_problem_sys(shape=(16, 8, 8), tau=1.0, seed=3)
    st = ctx.system_tensors(sysv)
    bh, s = st["bhat"].cpu().numpy(), st["s"].cpu().numpy()

    def spmv(x):
        y = torch.empty(ctx.n, dtype=torch.float64, device="cuda")
        ctx.spmv(torch.tensor(x, device="cuda"), y)
        return y.cpu().numpy()

    n = ctx.n
    r0 = bh - spmv(En.cpu().numpy() / s)
    z0 = np.maximum(r0, 0.0)
    q0 = spmv(z0)
    r1 = r0 - (r0 @ z0) / (z0 @ q0) * q0
    M0 = np.max(r0) * np.sqrt(n) / np.linalg.norm(r0)
    M1 = np.max(r1) * np.sqrt(n) / np.linalg.norm(r1)
    assert M1 > 1.15 * M0, (M0, M1)  # room for the bf16 rounding of the input and the gain
    gain = 3.39e38 / np.sqrt(M0 * M1)
    net = rt.Net(seed=1)
    net.set_params(_identity_path_params(gain, 1e-36))
    E = En.clone()
    rc, sl = ctx.solve(E, rt.solve_opts(rt.MODE_LEARNED, tol=1e-8, net=net, inner_max_iter=10, reduce=1),
                       raise_on_error=False)
    assert sl["precond_applies"] == 2, sl  # the first application was finite
    assert rc == rt.RT_OK and sl["fallback"] == 1 and sl["handover"] == 0 and sl["reduced"] == 1, sl
    assert sl["relres"] <= 1e-8
    assert np.all(np.isfinite(E.cpu().numpy()))
    E_f = En.clone()
    ctx.solve(E_f, rt.solve_opts(rt.MODE_FP64, tol=1e-10))
    Tl, Tf = T.clone(), T.clone()
    ctx.temperature(E, S, Tl)
    ctx.temperature(E_f, S, Tf)
    assert float(((Tl - Tf).abs() / Tf).max()) < 1e-5


def test_fgmres_reduced_finish_recovers_from_a_network_that_overflows_on_its_second_application():
    """Flexible GMRES with a network that is finite on the first Arnoldi vector and
    overflows on the second: the cycle ends before its update reaches y, the reduced
    finish starts from the previous iterate and meets the tolerance, and `fallback`
    reports the failed network.  The threshold lies between the largest entries of the
    two unit-RMS basis vectors, computed on the host from the GPU's assembled system
    (v_1 is A z_0 made orthogonal to v_0, z_0 proportional to relu(v_0)).  The system is
    one where the largest entry of v_1 exceeds that of v_0 (by a factor of about 1.9; on
    the 16 x 8 x 8 systems it is the other way round)."""
    from paper_1001_3301_amd import rt
    wl, ctx, rho, T, En, S, sysv = _small_problem_sys(shape=(32, 8, 8), tau=10.0, seed=7)
    st = ctx.system_tensors(sysv)
    bh, s = st["bhat"].cpu().numpy(), st["s"].cpu().numpy()

    def spmv(x):
        y = torch.empty(ctx.n, dtype=torch.float64, device="cuda")
        ctx.spmv(torch.tensor(x, device="cuda"), y)
        return y.cpu().numpy()

    n = ctx.n
    r0 = bh - spmv(En.cpu().numpy() / s)
    v0 = r0 / np.linalg.norm(r0)
    w = spmv(np.maximum(v0, 0.0))
    v1 = w - (w @ v0) * v0
    v1 /= np.linalg.norm(v1)
    M0, M1 = np.max(v0) * np.sqrt(n), np.max(v1) * np.sqrt(n)
    assert M1 > 1.15 * M0, (M0, M1)  # room for the bf16 rounding of the input and the gain
    net = rt.Net(seed=1)
    net.set_params(_identity_path_params(3.39e38 / np.sqrt(M0 * M1), 1e-36))
    E = En.clone()
    rc, sl = ctx.solve(E, rt.solve_opts(rt.MODE_LEARNED, tol=1e-8, net=net, inner_max_iter=10, reduce=1,
                                        inner=rt.INNER_FGMRES), raise_on_error=False)
    assert sl["precond_applies"] == 2, sl  # the first application was finite
    assert rc == rt.RT_OK and sl["fallback"] == 1 and sl["handover"] == 0 and sl["reduced"] == 1, sl
    assert sl["relres"] <= 1e-8
    assert np.all(np.isfinite(E.cpu().numpy()))


def test_residual_loss_gradient_against_oracle():
    """rt_net_loss_grad_resid (forward, A z with the fp32 operator, loss, A^T, backward)
    against the oracle's residual-loss gradient on the same bf16 weights and operator."""
    from paper_1001_3301_amd import rt
    shape = (16, 8, 8)
    n = 16 * 8 * 8
    wl, ctx = _ctx_for(shape)
    net = rt.Net(seed=5)
    p = net.get_params().astype(np.float64)
    pq = p.copy()
    for l, (taps, cout, cin) in enumerate(NN.layer_shapes()):
        o = NN.param_offset(l)
        nw = taps * cout * cin
        pq[o:o + nw] = bits_to_f64(bf16_bits(p[o:o + nw]))
    Xb = _net_input(n, 12)
    X64 = bits_to_f64(Xb).reshape(n, 16)
    g = _rng(13)
    r = g.standard_normal(n).astype(np.float32)
    a32 = (-0.16 * g.random(3 * n)).astype(np.float32)
    a32.reshape(3, 8, 8, 16)[0][:, :, -1] = 0.0
    a32.reshape(3, 8, 8, 16)[1][:, -1, :] = 0.0
    L_ref, g_ref, z_ref = NN.loss_grad_resid(shape, pq, X64, r.astype(np.float64), a32.astype(np.float64))
    z = torch.empty(n, dtype=torch.float32, device="cuda")
    L = net.loss_grad_resid(ctx, dev_bf16(Xb), dev_f32(r), dev_f32(a32), z)
    assert np.linalg.norm(z.cpu().numpy() - z_ref) <= 3e-2 * np.linalg.norm(z_ref)
    assert abs(L - L_ref) <= 3e-2 * L_ref
    gg = net.get_grads().astype(np.float64)
    # bf16 activations (relative rounding 2^-9 per layer) and ReLU masks taken from
    # them make the gradients of the layers far from the output differ from the float64
    # ones by up to ~15 % in norm on this input (direction within ~9 degrees)
    for l, (taps, cout, cin) in enumerate(NN.layer_shapes()):
        o = NN.param_offset(l)
        sl = slice(o, o + taps * cout * cin + cout)
        a, b = gg[sl], g_ref[sl]
        cos = np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300)
        assert cos > 0.98, (l, cos)
        assert np.linalg.norm(a - b) <= 0.2 * np.linalg.norm(b), l


def test_training_with_residual_loss_lowers_it():
    from paper_1001_3301_amd import rt
    wl, ctx, rho, T, En, S = _small_problem()
    ds = rt.Dataset(ctx, 8)
    ds.add(En, [0, 5, 20, 60])
    net = rt.Net(seed=11)
    st = net.train(ctx, ds, epochs=25, lr=2e-3, seed=1, loss=rt.LOSS_RESIDUAL)
    assert st["steps"] == 100
    assert st["loss_last_epoch"] < 0.7 * st["loss_first_epoch"], st


def test_what_the_trained_network_gains():
    """The trained preconditioner against the method without it, on an unseen field:
    per application it removes most of the residual that one Jacobi-CG step leaves, and
    after 10 iterations the learned flexible CG is well ahead of Jacobi CG; an untrained
    network of the same shape gains nothing.  (To a relative residual of 1e-8 the slow
    global modes dominate and the learned solve hands over to float64 CG: the budget and
    fallback keep it correct; the bench reports its wall time.)"""
    from paper_1001_3301_amd import rt
    shape = (64, 32, 32)
    rng = np.random.Generator(np.random.PCG64(21))
    wl0, ctx = _ctx_for(shape, n_nu=16, tau=1.0, seed=400)
    n = ctx.n

    def system(tau, seed):
        wl = sy.make_workload("t", *shape, 16, tau, seed)
        rho = torch.tensor(wl.rho.ravel(), device="cuda")
        T = torch.full((n,), wl.T_bc, dtype=torch.float64, device="cuda")
        q = torch.empty(n, dtype=torch.float64, device="cuda"); S = torch.empty_like(q)
        ctx.raytrace(rho, T, q, S)
        ctx.temperature(torch.full((n,), sy.A_RAD * wl.T_bc ** 4, dtype=torch.float64, device="cuda"), S, T)
        ctx.raytrace(rho, T, q, S)
        En = torch.empty_like(q)
        ctx.energy(T, S, En)
        ctx.assemble(rho, T, En, q)
        return En

    ds = rt.Dataset(ctx, 32)
    for f in range(8):
        ds.add(system(float(10 ** rng.uniform(-1, 2)), 410 + f), [0, 10, 40, 150])
    trained = rt.Net(seed=4)
    trained.train(ctx, ds, epochs=10, lr=1e-3, seed=1, loss=rt.LOSS_RESIDUAL)
    untrained = rt.Net(seed=4)
    En = system(10.0, 499)  # unseen field

    def relres_after(k, mode, net=None):
        E = En.clone()
        o = rt.solve_opts(mode, tol=1e-30, max_iter=k, inner_max_iter=k + 10, net=net)
        rc, st = ctx.solve(E, o, raise_on_error=False)
        assert rc in (rt.RT_OK, rt.RT_ENOCONV) and st["fallback"] == 0
        return st["relres"]

    cg1, cg10 = relres_after(1, rt.MODE_FP64), relres_after(10, rt.MODE_FP64)
    tr1, tr10 = relres_after(1, rt.MODE_LEARNED, trained), relres_after(10, rt.MODE_LEARNED, trained)
    un1 = relres_after(1, rt.MODE_LEARNED, untrained)
    print(f"relres after 1 / 10 iterations: Jacobi CG {cg1:.3e} / {cg10:.3e}, trained {tr1:.3e} / {tr10:.3e}, "
          f"untrained {un1:.3e}")
    assert tr1 < 0.5 * cg1 and tr1 < 0.5 * un1
    assert tr10 < 0.5 * cg10
    # the full solve stays correct and needs no more iterations than Jacobi CG alone
    E = En.clone()
    rc, sl = ctx.solve(E, rt.solve_opts(rt.MODE_LEARNED, tol=1e-8, net=trained, inner_max_iter=20))
    E = En.clone()
    rc, sf = ctx.solve(E, rt.solve_opts(rt.MODE_FP64, tol=1e-8))
    print(f"to 1e-8: learned (20 applications, then float64 CG) {sl['iters']} it, Jacobi CG {sf['iters']} it")
    assert sl["relres"] <= 1e-8 and sl["iters"] <= 1.1 * sf["iters"]


def test_learned_solve_with_reduced_mixed_finish():
    """reduce = 1 in the learned mode: after the network budget the reduced mixed solve
    finishes; the answer meets the tolerance and its temperature agrees with the float64
    solve's."""
    from paper_1001_3301_amd import rt
    wl, ctx, rho, T, En, S = _small_problem()
    assert ctx.shape[0] % 2 == 0 and ctx.shape[2] % 2 == 0
    net = rt.Net(seed=3)
    E = En.clone()
    rc, sl = ctx.solve(E, rt.solve_opts(rt.MODE_LEARNED, tol=1e-8, net=net, inner_max_iter=3, reduce=1))
    # the budget ran out: the planned hand-over, not a failure of the network
    assert sl["handover"] == 1 and sl["fallback"] == 0 and sl["reduced"] == 1 and sl["precond_applies"] == 3
    assert sl["relres"] <= 1e-8
    E_f = En.clone()
    rc, sf = ctx.solve(E_f, rt.solve_opts(rt.MODE_FP64, tol=1e-10))
    Tl, Tf = T.clone(), T.clone()
    ctx.temperature(E, S, Tl)
    ctx.temperature(E_f, S, Tf)
    assert float(((Tl - Tf).abs() / Tf).max()) < 1e-5


@pytest.mark.parametrize("inner", [0, 1], ids=["fcg", "fgmres"])
def test_learned_solves_against_the_oracle_dense_solve(inner):
    """The learned solve (float64 finish) and the learned solve with the reduced mixed
    finish, with a briefly trained network, against the oracle on 32 x 8 x 8: the
    oracle's own assembly and residual of the GPU's answer meet the tolerance, and the
    temperature from the GPU's E is within the reduced-precision bar (1e-3) of the
    oracle's dense (Cholesky) solve and Newton step (the measured error is printed)."""
    import oracle
    from paper_1001_3301_amd import rt
    shape = (32, 8, 8)
    wl, ctx, rho, T, En, S, sysv = _small_problem_sys(shape=shape, tau=10.0, seed=5)
    P = oracle.Problem.from_workload(wl)
    rh = wl.rho.ravel()
    To = np.full(P.n, wl.T_bc)
    _, So, _ = P.raytrace(rh, To, want_faces=False)
    To = P.newton(np.full(P.n, sy.A_RAD * wl.T_bc ** 4), So, To)
    qo, So, _ = P.raytrace(rh, To, want_faces=False)
    Eno = P.energy(To, So)
    out = P.assemble(rh, To, Eno, qo)
    E_ref = out["s"] * P.dense_solve(out["ahat"], out["bhat"])
    T_ref = P.newton(E_ref, So, To)
    ds = rt.Dataset(ctx, 4)
    ds.add(En, [0, 5, 20, 60])
    net = rt.Net(seed=6)
    net.train(ctx, ds, epochs=10, lr=1e-3, seed=1, loss=rt.LOSS_RESIDUAL)
    for reduce, budget in ((0, 20), (1, 5)):
        E = En.clone()
        rc, sl = ctx.solve(E, rt.solve_opts(rt.MODE_LEARNED, tol=1e-8, net=net, inner_max_iter=budget,
                                            reduce=reduce, inner=inner))
        assert rc == rt.RT_OK and sl["fallback"] == 0 and sl["precond_applies"] >= 1
        Eg = E.cpu().numpy()
        res = P.relres(out["ahat"], out["bhat"], Eg / out["s"])
        Tg = T.clone()
        ctx.temperature(E, S, Tg)
        eT = float(np.max(np.abs(Tg.cpu().numpy() - T_ref) / T_ref))
        eE = float(np.max(np.abs(Eg - E_ref) / np.abs(E_ref)))
        print(f"learned reduce={reduce}: {sl['precond_applies']} applications + {sl['iters']} iterations, "
              f"oracle relres {res:.3e}, T err {eT:.2e}, E err {eE:.2e} vs the oracle's dense solve")
        assert res <= 1.05e-8
        assert eT <= 1e-3


def _oracle_system(P, wl):
    """The oracle's assembled system of the first step from T_bc (the state
    _small_problem_sys prepares on the GPU)."""
    rh = wl.rho.ravel()
    To = np.full(P.n, wl.T_bc)
    _, So, _ = P.raytrace(rh, To, want_faces=False)
    To = P.newton(np.full(P.n, sy.A_RAD * wl.T_bc ** 4), So, To)
    qo, So, _ = P.raytrace(rh, To, want_faces=False)
    return P.assemble(rh, To, P.energy(To, So), qo)


def _linear_path_params(c):
    """Parameters of a network that maps its input channel 0 to c times itself: layer 0
    splits x into relu(x) and relu(-x) (channels 0 and 1), layers 1, 8 (from the skip
    connection) and 9 pass both on, the output layer takes c (relu(x) - relu(-x)) = c x.
    Every value it passes is a bf16 of the input times +-1, so its only error is the
    input's rounding to bf16: as a preconditioner it is c times the identity up to that
    rounding."""
    p = np.zeros(NN.param_count(), dtype=np.float32)
    centre = 13
    for l, co, ci, g in ((0, 0, 0, 1.0), (0, 1, 0, -1.0), (1, 0, 0, 1.0), (1, 1, 1, 1.0),
                         (8, 0, 32, 1.0), (8, 1, 33, 1.0), (9, 0, 0, 1.0), (9, 1, 1, 1.0)):
        taps, cout, cin = NN.layer_shapes()[l]
        p[NN.param_offset(l) + (centre * cout + co) * cin + ci] = g
    o = NN.param_offset(10)
    p[o + 0], p[o + 1] = c, -c
    return p


def test_fgmres_with_a_scaled_identity_network_converges_like_gmres():
    """Flexible GMRES(30) whose network is 3 x the identity (up to the bf16 rounding of its
    input) against plain GMRES(30) on the same system: the same convergence (within 25 %
    + 5 iterations), one application per iteration, no hand-over; the oracle's residual of
    the answer meets the tolerance.  The update must combine the preconditioned vectors
    Z: combining the Arnoldi basis instead would move y by a third of the step."""
    import oracle
    from paper_1001_3301_amd import rt
    shape = (32, 8, 8)
    wl, ctx, rho, T, En, S, sysv = _small_problem_sys(shape=shape, tau=10.0, seed=5)
    net = rt.Net(seed=1)
    net.set_params(_linear_path_params(3.0))
    r = _rng(41).standard_normal(ctx.n).astype(np.float32)
    z = torch.empty(ctx.n, dtype=torch.float32, device="cuda")
    net.apply(ctx, dev_f32(r), z)
    zr = z.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(zr - 3.0 * r)) <= 3.0 * 2.0 ** -8 * np.max(np.abs(r))
    E_g = En.clone()
    rc, sg = ctx.solve(E_g, rt.solve_opts(rt.MODE_GMRES, tol=1e-8, restart=30))
    E = En.clone()
    rc, sf = ctx.solve(E, rt.solve_opts(rt.MODE_LEARNED, tol=1e-8, net=net, inner_max_iter=100000, restart=30,
                                        inner=rt.INNER_FGMRES))
    print(f"GMRES(30) {sg['iters']} iterations; flexible GMRES(30) with 3 I: {sf['iters']} iterations, "
          f"{sf['precond_applies']} applications, relres {sf['relres']:.3e}")
    assert rc == rt.RT_OK and sf["handover"] == 0 and sf["fallback"] == 0
    assert sf["precond_applies"] == sf["iters"]
    assert sf["relres"] <= 1e-8
    assert sf["iters"] <= 1.25 * sg["iters"] + 5
    # the oracle's own residual of the GPU's answer, on the system the oracle assembles
    P = oracle.Problem.from_workload(wl)
    out = _oracle_system(P, wl)
    assert P.relres(out["ahat"], out["bhat"], E.cpu().numpy() / out["s"]) <= 1.05e-8


def test_fgmres_hands_over_when_the_budget_is_spent():
    """inner_max_iter = 3 network applications: the cycle is closed after three flexible
    GMRES steps and the planned finish (float64 CG; with reduce = 1 the reduced mixed
    solve) meets the tolerance."""
    from paper_1001_3301_amd import rt
    wl, ctx, rho, T, En, S = _small_problem()
    net = rt.Net(seed=3)
    for reduce in (0, 1):
        E = En.clone()
        rc, sl = ctx.solve(E, rt.solve_opts(rt.MODE_LEARNED, tol=1e-8, net=net, inner_max_iter=3, reduce=reduce,
                                            inner=rt.INNER_FGMRES))
        assert sl["handover"] == 1 and sl["fallback"] == 0 and sl["precond_applies"] == 3
        assert sl["relres"] <= 1e-8 and sl["reduced"] == reduce
        assert np.all(np.isfinite(E.cpu().numpy()))


def test_net_apply_is_the_scaled_forward_of_the_solver_input():
    """rt_net_apply: the input the learned solve builds (residual at unit RMS, the scaled
    operator's face features) through rt_net_forward, scaled back; positively homogeneous
    bit for bit (2 r gives exactly 2 z); no system, no application."""
    import oracle
    from paper_1001_3301_amd import rt
    from _util import initial_temperature
    shape = (16, 8, 8)
    n = 16 * 8 * 8
    wl, ctx = _ctx_for(shape)
    net = rt.Net(seed=11)
    r = _rng(21).standard_normal(n).astype(np.float32)
    z = torch.empty(n, dtype=torch.float32, device="cuda")
    with pytest.raises(rt.RtError) as ei:
        net.apply(ctx, dev_f32(r), z)
    assert ei.value.status == rt.RT_EINVAL
    P = oracle.Problem.from_workload(wl)
    T = initial_temperature(P, wl)
    q, S, _ = P.raytrace(wl.rho, T, want_faces=False)
    En = P.energy(T, S)
    ref = P.assemble(wl.rho, T, En, q)
    d64 = lambda x: torch.tensor(np.ascontiguousarray(x, dtype=np.float64).ravel(), device="cuda")
    ctx.assemble(d64(wl.rho), d64(T), d64(En), d64(q))
    net.apply(ctx, dev_f32(r), z)
    # the same input built on the host from the definition in rt.h
    s = np.sqrt(n / np.sum(r.astype(np.float64) ** 2))
    X = np.zeros((n, 16), dtype=np.float32)
    X[:, 0] = (r.astype(np.float64) * s).astype(np.float32)
    a = -ref["ahat"].reshape(3, n)
    with np.errstate(divide="ignore"):
        f = np.where(a > 1e-30, np.log10(np.maximum(a, 1e-300)), -30.0)
    X[:, 1:4] = ((np.clip(f, -30.0, 0.0) + 15.0) / 15.0).T.astype(np.float32)
    zf = torch.empty(n, dtype=torch.float32, device="cuda")
    net.forward(ctx, dev_bf16(bf16_bits(X.ravel())), zf)
    zref = (zf.cpu().numpy().astype(np.float64) / s).astype(np.float32)
    zg = z.cpu().numpy()
    assert np.all(np.isfinite(zg))
    assert np.linalg.norm(zg - zref) <= 1e-2 * np.linalg.norm(zref)
    z2 = torch.empty_like(z)
    net.apply(ctx, dev_f32(2.0 * r), z2)
    assert np.array_equal(z2.cpu().numpy(), 2.0 * zg)
