"""GPU parity of the BF16-MFMA refiner (forward, backward, features, apply)
against the oracle with identical bfloat16 rounding points."""
import numpy as np
import pytest

from oracle import convert as oc
from oracle import mlp as om
from paper_2502_07754_amd import scenes
from tests.helpers import gaussians_gpu

pytestmark = pytest.mark.gpu


def _params_gpu(p):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v.astype(np.float32))).cuda() for k, v in p.items()}


@pytest.mark.parametrize("N", [1, 37, 1000, 4099])
def test_forward_parity(gpu, N):
    import torch
    p = om.init_params(28, seed=N, zero_last=False)
    x = np.random.default_rng(N).normal(size=(N, 15)).astype(np.float32)
    x16 = np.concatenate([x, np.zeros((N, 1), np.float32)], 1)
    r = gpu.Refiner(28)
    r.set_weights(_params_gpu(p))
    y = r.forward(torch.from_numpy(x16).cuda()).cpu().numpy()
    ref, _ = om.forward(p, x.astype(np.float64))
    err = np.abs(y - ref).max()
    print("forward max err", err, "max |y|", np.abs(ref).max(), flush=True)
    assert err <= 1e-3 * np.abs(ref).max()


def test_forward_parity_persistent_grid(gpu):
    """Enough samples that every wavefront of the inference grid (one block
    per CU) takes several 32-sample groups, with a ragged last group: every
    row against the oracle. Rows agree to float32 accumulation order except
    where a hidden pre-activation lies so close to a bfloat16 rounding
    boundary that the float32 sum and the float64 sum round it to neighbouring
    bfloat16 values (one unit in the last place of one hidden unit, about 0.1%
    of rows): the bulk is held to 1e-6 of the output scale, the rare rows to a
    few such flips."""
    import torch
    N = 250_003
    p = om.init_params(28, seed=5, zero_last=False)
    x = np.random.default_rng(5).normal(size=(N, 15)).astype(np.float32)
    x16 = np.concatenate([x, np.zeros((N, 1), np.float32)], 1)
    r = gpu.Refiner(28)
    r.set_weights(_params_gpu(p))
    y = r.forward(torch.from_numpy(x16).cuda()).cpu().numpy()
    ref, _ = om.forward(p, x.astype(np.float64))
    e = np.abs(y - ref).max(1) / np.abs(ref).max()
    print("row error quantiles (50, 99, 99.9, max)", np.quantile(e, [0.5, 0.99, 0.999, 1.0]), flush=True)
    assert np.quantile(e, 0.99) <= 1e-6
    assert np.mean(e > 1e-5) <= 0.01
    assert e.max() <= 3e-3


def test_forward_rejects_unaligned_input(gpu):
    import torch
    from paper_2502_07754_amd._lib import MspError
    r = gpu.Refiner(28)
    r.set_weights(_params_gpu(om.init_params(28, seed=1, zero_last=False)))
    buf = torch.zeros(65 * 16, dtype=torch.float32, device="cuda")
    with pytest.raises(MspError, match="aligned"):
        r.forward(buf[1:1 + 64 * 16].view(64, 16))


@pytest.mark.parametrize("N", [50, 2048, 5000, 250_000])
def test_backward_parity(gpu, N):
    """Weight, bias and input gradients against the oracle at matching bfloat16
    rounding points; N = 250,000 is the training batch of the refiner workload
    (one epoch of the pair-training scenes)."""
    import torch
    p = om.init_params(28, seed=7 + N, zero_last=False)
    rng = np.random.default_rng(N)
    x = rng.normal(size=(N, 15)).astype(np.float32)
    dy = rng.normal(size=(N, 28)).astype(np.float32)
    x16 = np.concatenate([x, np.zeros((N, 1), np.float32)], 1)
    r = gpu.Refiner(28)
    r.set_weights(_params_gpu(p))
    g = r.backward(torch.from_numpy(x16).cuda(), torch.from_numpy(dy).cuda(), want_dx=True)
    _, cache = om.forward(p, x.astype(np.float64))
    ref = om.backward(p, cache, dy.astype(np.float64))
    dx = g.pop("x").cpu().numpy()
    assert dx.shape == (N, 16) and np.all(dx[:, 15] == 0)
    g["x"] = dx[:, :15]
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        a = g[k].cpu().numpy()
        err = np.abs(a - ref[k]).max()
        print(k, "max err", err, "max |g|", np.abs(ref[k]).max(), flush=True)
        assert err <= 1e-3 * np.abs(ref[k]).max(), k
    # the input gradient row by row: a row may miss the bar only where a hidden
    # unit's pre-activation sits within float32 rounding of its ReLU's kink (the
    # float32 sums may then take the other side, which switches that unit's whole
    # contribution); at most 0.5% of the rows may be such rows
    scale = np.abs(ref["x"]).max()
    row_err = np.abs(g["x"] - ref["x"]).max(axis=1)
    miss = np.flatnonzero(row_err > 1e-3 * scale)
    z1, z2 = om.preactivations(p, x.astype(np.float64))
    near = (np.abs(z1) <= 1e-5 * np.abs(z1).max()).any(axis=1) | (np.abs(z2) <= 1e-5 * np.abs(z2).max()).any(axis=1)
    print("x max err", row_err.max(), "max |g|", scale, "rows beyond the bar", len(miss),
          "rows with a unit at its kink", int(near.sum()), flush=True)
    assert np.all(near[miss]), miss[~near[miss]][:10]
    assert len(miss) <= 0.005 * N


def test_backward_reuses_its_buffers(gpu):
    """A larger backward, then a smaller one on other data with the same
    refiner: the second must not see the first's intermediates (the training
    buffer is cleared only where the kernels do not write)."""
    import torch
    p = om.init_params(28, seed=3, zero_last=False)
    r = gpu.Refiner(28)
    r.set_weights(_params_gpu(p))
    for N, seed in ((5000, 21), (1000, 22)):
        rng = np.random.default_rng(seed)
        x = rng.normal(size=(N, 15)).astype(np.float32)
        dy = rng.normal(size=(N, 28)).astype(np.float32)
        x16 = np.concatenate([x, np.zeros((N, 1), np.float32)], 1)
        g = r.backward(torch.from_numpy(x16).cuda(), torch.from_numpy(dy).cuda())
    _, cache = om.forward(p, x.astype(np.float64))
    ref = om.backward(p, cache, dy.astype(np.float64))
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        a = g[k].cpu().numpy()
        assert np.abs(a - ref[k]).max() <= 1e-3 * np.abs(ref[k]).max(), k


def test_backward_weight_gradients_repeat_exactly(gpu):
    """Weight and bias gradients are summed in a fixed order (no float
    atomics): two identical backwards give identical bits."""
    import torch
    p = om.init_params(28, seed=9, zero_last=False)
    r = gpu.Refiner(28)
    r.set_weights(_params_gpu(p))
    rng = np.random.default_rng(9)
    N = 20_000
    x16 = np.concatenate([rng.normal(size=(N, 15)), np.zeros((N, 1))], 1).astype(np.float32)
    dy = rng.normal(size=(N, 28)).astype(np.float32)
    xg, dg = torch.from_numpy(x16).cuda(), torch.from_numpy(dy).cuda()
    g1 = {k: v.cpu().numpy() for k, v in r.backward(xg, dg).items()}
    g2 = {k: v.cpu().numpy() for k, v in r.backward(xg, dg).items()}
    for k in ("W1", "W2", "W3", "b1", "b2", "b3"):
        assert np.array_equal(g1[k], g2[k]), k


def test_forward_bf16_rounding_bitwise(gpu):
    """Unit weights W1[0][0] = W2[0][0] = W3[0][0] = 1 (all else zero) pass
    input feature 0 through the forward's three bfloat16 roundings unchanged
    after the first, so output 0 is bf16(x0) for x0 >= 0: ties with even and
    odd last bits, their neighbours one float32 ulp away, random low bits and
    exact bfloat16 values, bit for bit against the oracle's rounding (positive
    normal values; the matrix core may flush subnormals)."""
    import torch
    n_out = 28
    p = {k: np.zeros_like(v) for k, v in om.init_params(n_out, seed=0, zero_last=False).items()}
    p["W1"][0, 0] = p["W2"][0, 0] = p["W3"][0, 0] = 1.0
    rng = np.random.default_rng(0)
    hi = rng.integers(0x0080, 0x7F00, 2000).astype(np.uint32) << 16  # sign 0, exponent 1..253
    tie = hi | 0x8000
    bits = np.concatenate([tie, tie + 1, tie - 1, hi | rng.integers(0, 0x10000, 2000).astype(np.uint32), hi])
    x0 = bits.view(np.float32)
    assert np.all(np.isfinite(x0)) and np.all(x0 > 0)
    N = len(x0)
    x16 = np.zeros((N, 16), np.float32)
    x16[:, 0] = x0
    r = gpu.Refiner(n_out)
    r.set_weights(_params_gpu(p))
    y = r.forward(torch.from_numpy(x16).cuda()).cpu().numpy()
    want = om.bf16_round(x0)
    assert np.array_equal(y[:, 0].astype(np.float64), want)
    assert np.all(y[:, 1:] == 0)


def test_empty_batch(gpu):
    """No samples: the forward returns no rows, the backward zero gradients."""
    import torch
    p = om.init_params(28, seed=4, zero_last=False)
    r = gpu.Refiner(28)
    r.set_weights(_params_gpu(p))
    x = torch.zeros((0, 16), dtype=torch.float32, device="cuda")
    dy = torch.zeros((0, 28), dtype=torch.float32, device="cuda")
    assert r.forward(x).shape == (0, 28)
    g = r.backward(x, dy, want_dx=True)
    assert g["x"].shape == (0, 16)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        assert torch.count_nonzero(g[k]).item() == 0, k


def test_features_and_apply(gpu):
    g = scenes.gaussians(500, 4, 0.01, 0.1, flat=True)
    gg = gaussians_gpu(g)
    x = gpu.refiner_features(gg, 8).cpu().numpy()
    ref = om.features(g.mean, g.scale, g.quat, g.opacity, g.rgb, 8)
    np.testing.assert_allclose(x[:, :15], ref, rtol=1e-6, atol=1e-7)
    assert np.all(x[:, 15] == 0)
    import torch
    y = np.random.default_rng(1).normal(0, 0.05, (500, 28)).astype(np.float32)
    out = gpu.refiner_apply(gg, 8, 2.0, torch.from_numpy(y).cuda())
    want = om.refined_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, 8, 2.0, y.astype(np.float64))
    np.testing.assert_array_equal(out["idx"].cpu().numpy(), want["idx"])
    np.testing.assert_allclose(out["pos"].cpu().numpy(), want["pos"], atol=2e-6)
    np.testing.assert_allclose(out["opacity"].cpu().numpy(), want["opacity"], atol=1e-6)
    np.testing.assert_allclose(out["rgb"].cpu().numpy(), want["rgb"], atol=1e-6)
    # zero corrections reproduce the plain conversion
    z = gpu.refiner_apply(gg, 8, 2.0, torch.zeros((500, 28), device="cuda"))
    plain = oc.convert_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, 8, 2.0)
    np.testing.assert_allclose(z["pos"].cpu().numpy(), plain["pos"], atol=2e-6)


def test_targets_and_loss(gpu):
    import torch
    from tests.helpers import faces_f32, to_gpu
    g = scenes.gaussians(400, 5, 0.01, 0.1, flat=True)
    K = 8
    rng = np.random.default_rng(3)
    y = rng.normal(0, 0.1, (400, 3 * K + 4))
    y[:, 3 * K] = rng.uniform(-0.05, 0.05, 400) * np.asarray(g.opacity)
    tuned = faces_f32(om.refined_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, K, 2.0, y))
    got = gpu.refiner_targets(gaussians_gpu(g), K, 2.0, to_gpu(tuned)).cpu().numpy()
    ref = om.fit_targets(g.mean, g.scale, g.quat, g.opacity, g.rgb, K, 2.0,
                         {k: v.astype(np.float64) if v.dtype == np.float32 else v for k, v in tuned.items()})
    np.testing.assert_allclose(got, ref, atol=2e-4)
    np.testing.assert_allclose(got, y, atol=5e-4)
    r = gpu.Refiner(3 * K + 4)
    a = torch.from_numpy(rng.normal(size=(400, 28)).astype(np.float32)).cuda()
    b = torch.from_numpy(rng.normal(size=(400, 28)).astype(np.float32)).cuda()
    L, dy = gpu.refiner_loss(r, a, b)
    d = (a - b).double().cpu().numpy()
    assert float(L.item()) == pytest.approx(np.mean(d * d), rel=1e-5)
    np.testing.assert_allclose(dy.cpu().numpy(), 2 * d / d.size, rtol=1e-5, atol=1e-9)


def test_weights_and_weighted_loss(gpu):
    import torch
    K = 8
    g = scenes.gaussians(300, 12, 0.01, 0.1, flat=True)
    w = gpu.refiner_weights(gaussians_gpu(g), K, 2.0, 0.1)
    ref = om.loss_weights(g.scale, K, 2.0, 0.1)
    np.testing.assert_allclose(w.cpu().numpy(), ref, rtol=2e-6)
    rng = np.random.default_rng(4)
    r = gpu.Refiner(3 * K + 4)
    a = rng.normal(size=(300, 3 * K + 4)).astype(np.float32)
    b = rng.normal(size=(300, 3 * K + 4)).astype(np.float32)
    # the weighted loss takes the oracle's weights (float32) on both sides
    w32 = ref.astype(np.float32)
    L, dy = gpu.refiner_loss(r, torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), torch.from_numpy(w32).cuda())
    rl, rg = om.weighted_mse(a, b, w32.astype(np.float64))
    assert float(L.item()) == pytest.approx(rl, rel=1e-5)
    np.testing.assert_allclose(dy.cpu().numpy(), rg, rtol=1e-5, atol=1e-12)


def test_apply_backward_parity(gpu):
    import torch
    K = 8
    g = scenes.gaussians(500, 14, 0.01, 0.1, flat=True)
    rng = np.random.default_rng(9)
    y = rng.normal(0, 0.2, (500, 3 * K + 4)).astype(np.float32)
    y[:, 3 * K] = rng.uniform(-0.2, 0.2, 500)
    V = 500 * (K + 1)
    gr = {k: rng.normal(size=sh).astype(np.float32) for k, sh in
          (("dpos", (3, V)), ("dopacity", (V,)), ("drgb", (3, V)))}
    got = gpu.refiner_apply_backward(gaussians_gpu(g), K, 2.0, torch.from_numpy(y).cuda(),
                                     {k: torch.from_numpy(v).cuda() for k, v in gr.items()}).cpu().numpy()
    ref = om.refined_fan_backward(g.mean, g.scale, g.quat, g.opacity, g.rgb, K, 2.0, y, gr["dpos"], gr["dopacity"],
                                  gr["drgb"])
    np.testing.assert_allclose(got, ref, rtol=1e-4, atol=1e-5 * np.abs(ref).max())


def test_refiner_pairs_and_supervised_training(gpu):
    """Pairs from the method's own fine-tuning; supervised training on them
    (MFMA forward/backward, weighted loss) lowers its loss."""
    from paper_2502_07754_amd import refiner_train as rt
    x, ys, w = rt.make_pairs(range(1000, 1003), n=2000, steps=60, res=64)
    assert x.shape[0] == 6000 and ys.shape == (6000, 28) and w.shape == (6000, 28)
    R, p, hist = rt.train(x, ys, w, steps=200, lr=3e-3)
    assert hist[-1][1] < hist[0][1], hist


def test_refiner_training_gains_on_heldout(gpu):
    """Trained on the fine-tuning objective of a few small scenes (render adjoint
    -> refiner_apply adjoint -> MFMA backward), the refiner's fans start closer
    to the targets of held-out scenes than the plain conversion's."""
    from paper_2502_07754_amd import refiner_train as rt
    data = rt.scene_data(range(1000, 1004), n=3000, res=96)
    R, p, hist = rt.train_image(data, steps=300, lr=1e-3)
    ev = rt.evaluate(R, [2000, 2001], n=3000, res=96)
    print(hist, ev, flush=True)
    assert all(e["refined"] < e["plain"] for e in ev), ev
