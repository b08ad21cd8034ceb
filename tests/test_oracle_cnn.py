"""Pins of the FP64 network oracle (oracle/cnn.py) to things other than itself: a library
correlation, adjoint identities, finite differences, torch's bfloat16 rounding and torch's
Adam. CPU only."""
import numpy as np
import pytest
import scipy.ndimage as ndi
import torch

from oracle import cnn
from paper_2404_03313_amd import synth


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def test_param_count_and_layout():
    # 27*1*32+32 + 3*(27*32*32+32) + 27*32*1+1
    assert cnn.param_count() == 84801
    p = np.arange(cnn.param_count(), dtype=np.float64)
    layers = cnn.unpack(p)
    assert [W.shape for W, _ in layers] == [(27, 32, 1), (27, 32, 32), (27, 32, 32), (27, 32, 32),
                                            (27, 1, 32)]
    assert layers[0][1][0] == 27 * 32 and layers[4][1][0] == cnn.param_count() - 1
    np.testing.assert_array_equal(cnn.pack(layers), p)


def test_bf16_round_matches_torch():
    rng = _rng(1)
    x = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e-3, 2000), [0.0, -0.0]])
    # exact ties: 1 + 2^-8 -> 1 (even), 1 + 3*2^-8 -> 1 + 2^-6 (even), -(1 + 2^-8) -> -1
    ties = np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 2 + 2 ** -7])
    np.testing.assert_array_equal(cnn.bf16_round(ties), [1.0, 1 + 2 ** -6, -1.0, 2.0])
    x = np.concatenate([x, ties])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cnn.bf16_round(x), ref)


@pytest.mark.parametrize("shape", [(2, 4, 5, 6), (1, 1, 3, 7), (3, 2, 2, 2)])
def test_conv_matches_scipy_correlate_per_volume(shape):
    """Each output channel is the bias plus, over the input channels, the zero-padded 3x3x3
    correlation (scipy.ndimage.correlate), taken per volume so no volume sees another."""
    rng = _rng(2)
    nb = shape[0]
    cin, cout = 3, 2
    x = rng.normal(size=shape + (cin,))
    W = rng.normal(size=(27, cout, cin))
    b = rng.normal(size=cout)
    y = cnn.conv(x, W, b)
    for vol in range(nb):
        for co in range(cout):
            ref = b[co] + sum(
                ndi.correlate(x[vol, ..., ci], W[:, co, ci].reshape(3, 3, 3), mode="constant", cval=0.0)
                for ci in range(cin))
            np.testing.assert_allclose(y[vol, ..., co], ref, rtol=1e-12, atol=1e-12)


def test_conv_adj_is_the_adjoint():
    rng = _rng(3)
    x = rng.normal(size=(2, 3, 4, 5, 4))
    g = rng.normal(size=(2, 3, 4, 5, 3))
    W = rng.normal(size=(27, 3, 4))
    lhs = np.sum(cnn.conv(x, W, np.zeros(3)) * g)
    rhs = np.sum(x * cnn.conv_adj(g, W))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_conv_wgrad_is_the_weight_derivative():
    """<g, conv(x, dW, db)> is linear in (dW, db) with coefficients conv_wgrad(x, g)."""
    rng = _rng(4)
    x = rng.normal(size=(2, 3, 4, 5, 4))
    g = rng.normal(size=(2, 3, 4, 5, 3))
    gw, gb = cnn.conv_wgrad(x, g)
    for trial in range(3):
        dW = rng.normal(size=(27, 3, 4))
        db = rng.normal(size=3)
        lhs = np.sum(g * cnn.conv(x, dW, db))
        rhs = np.sum(gw * dW) + np.sum(gb * db)
        assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1.0)


def _loss(params, v, target):
    return cnn.loss_grad(params, v, target, "exact")[0]


def test_loss_gradient_by_central_differences():
    """Directional derivatives of the exact loss along random directions restricted to each
    layer's weights and biases match central differences (so a dropped term, a wrong sign or a
    transposed operand in any layer's backward fails)."""
    rng = _rng(5)
    v = rng.uniform(size=(2, 3, 4, 5))
    target = v + rng.normal(0, 0.1, size=v.shape)
    params = synth.cnn_random_params(seed=6).astype(np.float64)
    loss, grad = cnn.loss_grad(params, v, target, "exact")
    n = cnn.param_count()
    off = 0
    for ci, co in cnn.layer_sizes():
        for part, size in (("W", 27 * co * ci), ("b", co)):
            d = np.zeros(n)
            d[off:off + size] = rng.normal(size=size)
            off += size
            h = 1e-6
            fd = (_loss(params + h * d, v, target) - _loss(params - h * d, v, target)) / (2 * h)
            an = float(grad @ d)
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-8), (ci, co, part, fd, an)
    assert off == n


def test_zero_network_is_identity_and_mse():
    """With every parameter zero, u0 = v and the loss is the plain mean squared error."""
    rng = _rng(7)
    v = rng.uniform(size=(1, 3, 3, 4))
    target = rng.uniform(size=v.shape)
    params = np.zeros(cnn.param_count())
    u, _ = cnn.forward(params, v)
    np.testing.assert_array_equal(u, v)
    loss, grad = cnn.loss_grad(params, v, target)
    assert loss == pytest.approx(np.mean((v - target) ** 2), rel=1e-15)
    # only the last bias sees a gradient (all hidden activations are zero)
    assert np.count_nonzero(grad) == 1
    assert grad[-1] == pytest.approx(2 * np.mean(v - target), rel=1e-12)


def test_receptive_field_is_five_voxels():
    """u0 at a voxel depends only on v within distance 5 per axis: the output at the centre of
    an 11^3 crop equals the full-volume output (what the full-size sampled GPU check uses)."""
    rng = _rng(8)
    v = rng.uniform(size=(1, 14, 13, 15))
    params = synth.cnn_random_params(seed=9).astype(np.float64)
    u, _ = cnn.forward(params, v)
    for (i, j, b) in [(7, 6, 7), (2, 3, 12), (0, 0, 0), (13, 12, 14)]:
        lo = [max(c - 5, 0) for c in (i, j, b)]
        hi = [min(c + 6, n) for c, n in zip((i, j, b), v.shape[1:])]
        crop = v[:, lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        uc, _ = cnn.forward(params, crop)
        assert uc[0, i - lo[0], j - lo[1], b - lo[2]] == pytest.approx(u[0, i, j, b], abs=1e-13)


def test_adam_matches_torch_optimizer():
    rng = _rng(10)
    p0 = rng.normal(size=50)
    grads = [rng.normal(size=50) for _ in range(4)]
    pt = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v2 = p0.copy(), np.zeros(50), np.zeros(50)
    for k, g in enumerate(grads, start=1):
        pt.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v2 = cnn.adam(p, m, v2, g, k, 1e-3)
    np.testing.assert_allclose(p, pt.detach().numpy(), rtol=0, atol=1e-14)


# ------------------------------------------------ the storage-rounding bound of the GPU tests

def _bound_inputs(shape, seed):
    rng = _rng(seed)
    v = rng.uniform(0, 1, size=shape).astype(np.float32).astype(np.float64)
    target = (v + rng.normal(0, 0.05, size=shape)).astype(np.float32).astype(np.float64)
    return v, target


def test_storage_rounding_bound_covers_bf16_rounding():
    """The bound the GPU tests apply against the exact network (LAMBDA x the spread of random
    bfloat16-sized relative errors at the storage points) holds for the actual round-to-nearest
    bfloat16 errors at those points (the oracle's bf16 mode), for the output and every
    parameter block, with the deterministic error of the size the random model predicts."""
    import cnn_error_bound as eb
    v, target = _bound_inputs((2, 7, 9, 21), 71)
    params = synth.cnn_random_params(seed=72).astype(np.float64)
    u0, spread = eb.forward_spread(params, v)
    ub, _ = cnn.forward(params, v, "bf16")
    r = np.linalg.norm(ub - u0) / spread
    assert 0.1 < r < eb.LAMBDA, r
    loss, g, sp, sp_loss = eb.grad_spread(params, v, target)
    lb, gb = cnn.loss_grad(params, v, target, "bf16")
    assert abs(lb - loss) <= eb.LAMBDA * sp_loss
    for name, a, b in eb.blocks():
        r = np.linalg.norm(gb[a:b] - g[a:b]) / sp[name]
        assert 0.05 < r < eb.LAMBDA, (name, r)
        # the bound is a small fraction of the gradient itself
        assert sp[name] < 0.05 * np.linalg.norm(g[a:b]), name


def test_storage_rounding_bound_rejects_planted_mistakes():
    """Structural mistakes in a network that rounds where the kernels round exceed the bound:
    one tap of a middle layer read mirrored (forward), and the sign of one hidden layer's data
    gradient lost in the backward pass (gradient)."""
    import cnn_error_bound as eb
    v, target = _bound_inputs((2, 7, 9, 21), 73)
    params = synth.cnn_random_params(seed=74).astype(np.float64)
    u0, spread = eb.forward_spread(params, v)
    layers = cnn.unpack(params)
    W = layers[2][0].copy()
    W[[0, 26]] = W[[26, 0]]          # tap (-1,-1,-1) swapped with (+1,+1,+1)
    layers[2] = (W, layers[2][1])
    bad, _ = cnn.forward(cnn.pack(layers), v, "bf16")
    assert np.linalg.norm(bad - u0) > 10 * eb.LAMBDA * spread

    loss, g, sp, _ = eb.grad_spread(params, v, target)
    orig = cnn.conv_adj
    calls = {"n": 0}

    def adj_unmasked(gg, Wt):
        # the second data gradient of the backward pass loses its sign
        calls["n"] += 1
        out = orig(gg, Wt)
        return out if calls["n"] != 2 else np.abs(out)
    cnn.conv_adj = adj_unmasked
    try:
        _, gbad = cnn.loss_grad(params, v, target, "bf16")
    finally:
        cnn.conv_adj = orig
    worst = max(np.linalg.norm(gbad[a:b] - g[a:b]) / sp[n] for n, a, b in eb.blocks())
    assert worst > 10 * eb.LAMBDA
