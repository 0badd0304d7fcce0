"""rt_nn_conv3d_bwd_weight_noalloc (partial sums in a static device array, no allocation)
against rt_nn_conv3d_bwd_weight (partial sums in a buffer allocated per call): the same
kernels, so the weight and bias gradients must agree bit for bit, on two calls in a row,
the second on a smaller grid with other channel counts (the array keeps the first call's
partial sums, which the second must overwrite before reading).  Layers wider than the
array are refused on the host."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _bf16_dev(x):
    return torch.tensor(np.asarray(x, dtype=np.float32)).to(torch.bfloat16).cuda()


def _case(shape, c1, up1, c2, cout, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    nr, nt, npp = shape
    n = nr * nt * npp
    n1 = n // 8 if up1 else n
    return dict(
        shape=shape, c1=c1, up1=up1, c2=c2, cout=cout,
        dy=torch.tensor(g.standard_normal(n * cout).astype(np.float32), device="cuda"),
        yr=_bf16_dev(g.standard_normal(n * cout)),
        x1=_bf16_dev(g.standard_normal(n1 * c1)),
        x2=_bf16_dev(g.standard_normal(n * c2)) if c2 else None,
    )


def _grads(case, noalloc):
    from paper_1001_3301_amd import rt
    cout, cin = case["cout"], case["c1"] + case["c2"]
    dw = torch.full((27 * cout * cin,), float("nan"), dtype=torch.float32, device="cuda")
    db = torch.full((cout,), float("nan"), dtype=torch.float32, device="cuda")
    rt.nn_conv_bwd_weight(case["shape"], case["dy"], case["yr"], cout, case["x1"], case["c1"], case["up1"],
                          case["x2"], case["c2"], dw, db, noalloc=noalloc)
    torch.cuda.synchronize()
    return dw.cpu().numpy(), db.cpu().numpy()


def test_noalloc_weight_gradient_equals_the_allocating_entry_point():
    first = _case((64, 64, 32), 16, 0, 0, 16, 1)     # 1024 tiles: 256 blocks of partial sums
    second = _case((16, 8, 8), 32, 1, 16, 16, 2)     # smaller grid, three input slices
    for case in (first, second):
        dw_a, db_a = _grads(case, noalloc=False)
        dw_b, db_b = _grads(case, noalloc=True)
        assert np.all(np.isfinite(dw_b)) and np.all(np.isfinite(db_b))
        assert np.array_equal(dw_a, dw_b) and np.array_equal(db_a, db_b), case["shape"]


def test_noalloc_refuses_layers_wider_than_its_scratch():
    from paper_1001_3301_amd import rt
    case = _case((64, 64, 32), 64, 0, 0, 64, 3)  # 256 blocks x 27 x 64 x 64 floats > 8 Mi
    dw = torch.empty(27 * 64 * 64, dtype=torch.float32, device="cuda")
    db = torch.empty(64, dtype=torch.float32, device="cuda")
    with pytest.raises(rt.RtError, match="static scratch"):
        rt.nn_conv_bwd_weight(case["shape"], case["dy"], case["yr"], 64, case["x1"], 64, 0, None, 0, dw, db,
                              noalloc=True)
