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


@pytest.mark.parametrize("case", CONV_CASES, ids=[str(c) for c in CONV_CASES])
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


@pytest.mark.parametrize("case", CONV_CASES, ids=[str(c) for c in CONV_CASES])
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
    from paper_1001_3301_amd import rt
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
    ctx.assemble(rho, T, En, q)
    return wl, ctx, rho, T, En, S


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


def test_learned_solve_falls_back_when_the_network_blows_up():
    from paper_1001_3301_amd import rt
    wl, ctx, rho, T, En, S = _small_problem(shape=(16, 8, 8))
    net = rt.Net(seed=2)
    p = net.get_params()
    net.set_params(np.full_like(p, 1e30))  # finite weights, overflowing activations
    E = En.clone()
    rc, st = ctx.solve(E, rt.solve_opts(rt.MODE_LEARNED, tol=1e-8, net=net))
    assert st["fallback"] == 1 and st["relres"] <= 1e-8
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
    assert sl["fallback"] == 1 and sl["reduced"] == 1 and sl["precond_applies"] == 3
    assert sl["relres"] <= 1e-8
    E_f = En.clone()
    rc, sf = ctx.solve(E_f, rt.solve_opts(rt.MODE_FP64, tol=1e-10))
    Tl, Tf = T.clone(), T.clone()
    ctx.temperature(E, S, Tl)
    ctx.temperature(E_f, S, Tf)
    assert float(((Tl - Tf).abs() / Tf).max()) < 1e-5


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
