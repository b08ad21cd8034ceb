"""GPU parity of the initial-estimate network (s3ttv_cnn_*) against the FP64 oracle in its
bf16 mode (same rounding points as the kernels, FP64 sums).

Tolerances. The remaining difference is the FP32 summation order of the kernels (relative
~1e-6 of the summed magnitudes) and, through it, rare one-ulp BF16 rounding flips of stored
activations or gradients (one ulp = 2^-8 relative, at a rate of roughly FP32 error / BF16 ulp
~ 1e-4 of the stored values). Both are far below a BF16 ulp in aggregate, so:
  * forward:  ||du0|| <= 2e-4 ||f|| (f = u0 - v) and max |du0| <= 2e-3 max |f|;
  * gradient: per layer block (weights, biases) ||dg|| <= 1e-3 ||g||;
  * Adam:     the update, per block, ||dupdate|| <= 1e-3 ||update||.
A systematic error (a wrong tap, a lost ReLU mask, truncation instead of rounding to
nearest) moves every value by a BF16 ulp or more and fails these bounds.

The same kernels are also compared with the exact FP64 network (the oracle's exact mode), under
a bound that follows from the storage formats alone (tests/cnn_error_bound.py): LAMBDA = 3 times
the spread of independent relative errors of bfloat16 size at the storage points. That check
does not depend on the oracle's bf16 mode choosing the same rounding points as the kernels.
"""
import numpy as np
import pytest
import torch

from oracle import cnn
from paper_2404_03313_amd import native as nt
from paper_2404_03313_amd import synth

pytestmark = pytest.mark.gpu

SHAPES = [(2, 7, 9, 21), (1, 1, 1, 1), (1, 1, 5, 3), (3, 5, 4, 17), (1, 16, 16, 16)]


def _inputs(shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.uniform(0, 1, size=shape).astype(np.float32)
    target = (v + rng.normal(0, 0.05, size=shape)).astype(np.float32)
    return v, target


def _blocks():
    off = 0
    for ci, co in cnn.layer_sizes():
        yield f"W{ci}->{co}", off, off + 27 * ci * co
        off += 27 * ci * co
        yield f"b{ci}->{co}", off, off + co
        off += co


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_matches_oracle(device, shape):
    print(f"forward shape={shape}", flush=True)
    v, _ = _inputs(shape, 11)
    params = synth.cnn_random_params(seed=12)
    u0 = nt.cnn_forward(torch.from_numpy(params).to(device), torch.from_numpy(v).to(device))
    torch.cuda.synchronize()
    got = u0.cpu().numpy().astype(np.float64)
    ref, _ = cnn.forward(params.astype(np.float64), v.astype(np.float64), "bf16")
    f_ref = ref - v
    err = got - ref
    print(f"  rel L2 {np.linalg.norm(err) / np.linalg.norm(f_ref):.2e} "
          f"max {np.abs(err).max() / np.abs(f_ref).max():.2e}", flush=True)
    assert np.linalg.norm(err) <= 2e-4 * np.linalg.norm(f_ref)
    assert np.abs(err).max() <= 2e-3 * np.abs(f_ref).max()


@pytest.mark.parametrize("shape", [(2, 7, 9, 21), (1, 1, 5, 3), (3, 5, 4, 17)])
def test_gradient_matches_oracle(device, shape):
    print(f"gradient shape={shape}", flush=True)
    v, target = _inputs(shape, 21)
    params = synth.cnn_random_params(seed=22)
    loss, grad = nt.cnn_grad(torch.from_numpy(params).to(device), torch.from_numpy(v).to(device),
                             torch.from_numpy(target).to(device))
    g = grad.cpu().numpy().astype(np.float64)
    rl, rg = cnn.loss_grad(params.astype(np.float64), v.astype(np.float64),
                           target.astype(np.float64), "bf16")
    assert loss == pytest.approx(rl, rel=1e-4)
    for name, a, b in _blocks():
        e = _rel(g[a:b], rg[a:b])
        print(f"  {name}: rel L2 {e:.2e}", flush=True)
        assert e <= 1e-3, name


def test_train_step_matches_oracle_adam(device):
    shape = (2, 7, 9, 21)
    v, target = _inputs(shape, 31)
    params = synth.cnn_random_params(seed=32).astype(np.float64)
    _, rg = cnn.loss_grad(params, v.astype(np.float64), target.astype(np.float64), "bf16")
    # moments from earlier steps: m ~ gradient-sized noise, second moment ~ 10 x the block's
    # mean square gradient, so the update is a smooth function of the gradient
    rng = np.random.Generator(np.random.PCG64(33))
    m0 = np.empty_like(params)
    v0 = np.empty_like(params)
    for _, a, b in _blocks():
        rms = np.sqrt(np.mean(rg[a:b] ** 2))
        m0[a:b] = rng.normal(0, rms, size=b - a)
        v0[a:b] = 10 * rms ** 2 * rng.uniform(0.5, 2.0, size=b - a)
    m0, v0 = m0.astype(np.float32), v0.astype(np.float32)
    p32 = params.astype(np.float32)
    step, lr = 3, 0.1
    tp, tm, tv = (torch.from_numpy(x.copy()).to(device) for x in (p32, m0, v0))
    nt.cnn_train_step(tp, tm, tv, step, lr, torch.from_numpy(v).to(device),
                      torch.from_numpy(target).to(device))
    rp, rm, rv = cnn.adam(p32.astype(np.float64), m0.astype(np.float64), v0.astype(np.float64), rg,
                          step, lr)
    gp, gm = tp.cpu().numpy().astype(np.float64), tm.cpu().numpy().astype(np.float64)
    for name, a, b in _blocks():
        du_gpu = gp[a:b] - p32[a:b]
        du_ref = rp[a:b] - p32[a:b]
        e = _rel(du_gpu, du_ref)
        print(f"  {name}: update rel L2 {e:.2e}", flush=True)
        assert e <= 1e-3, name
        assert _rel(gm[a:b], rm[a:b]) <= 1e-3, name
    assert _rel(tv.cpu().numpy().astype(np.float64), rv) <= 1e-5


def test_results_are_reproducible(device):
    shape = (3, 5, 4, 17)
    v, target = _inputs(shape, 41)
    params = torch.from_numpy(synth.cnn_random_params(seed=42)).to(device)
    tv, tt = torch.from_numpy(v).to(device), torch.from_numpy(target).to(device)
    l1, g1 = nt.cnn_grad(params, tv, tt)
    l2, g2 = nt.cnn_grad(params, tv, tt)
    assert l1 == l2 and torch.equal(g1, g2)
    assert torch.equal(nt.cnn_forward(params, tv), nt.cnn_forward(params, tv))


def test_stacked_volumes_are_independent(device):
    """A stack of volumes gives exactly the results of the volumes run one by one."""
    shape = (3, 5, 4, 17)
    v, _ = _inputs(shape, 51)
    params = torch.from_numpy(synth.cnn_random_params(seed=52)).to(device)
    tv = torch.from_numpy(v).to(device)
    stacked = nt.cnn_forward(params, tv)
    for k in range(shape[0]):
        assert torch.equal(stacked[k], nt.cnn_forward(params, tv[k].contiguous()))


def test_forward_full_scene_sampled(device):
    """The 512 x 512 x 191 scene of the warm-start measurement: u0 at sampled voxels (corners,
    faces, interior) against the oracle on the 11^3 crop that holds each voxel's receptive
    field."""
    cfg = synth.WORKLOADS["c5"]["cfg"]
    print(f"full scene {cfg.n1}x{cfg.n2}x{cfg.n3}", flush=True)
    v = synth.make_hsi(cfg)["v"]
    params = synth.cnn_random_params(seed=62)
    u0 = nt.cnn_forward(torch.from_numpy(params).to(device), torch.from_numpy(v).to(device))
    got = u0.cpu().numpy()
    n = v.shape
    rng = np.random.Generator(np.random.PCG64(63))
    pts = [(0, 0, 0), (n[0] - 1, n[1] - 1, n[2] - 1), (0, n[1] - 1, 95), (n[0] - 1, 0, 0),
           (255, 0, 190), (3, 300, 1)]
    pts += [tuple(int(rng.integers(0, m)) for m in n) for _ in range(18)]
    p64 = params.astype(np.float64)
    errs, fs = [], []
    for (i, j, b) in pts:
        lo = [max(c - 5, 0) for c in (i, j, b)]
        hi = [min(c + 6, m) for c, m in zip((i, j, b), n)]
        crop = v[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]].astype(np.float64)
        ref, _ = cnn.forward(p64, crop, "bf16")
        r = ref[i - lo[0], j - lo[1], b - lo[2]]
        errs.append(abs(float(got[i, j, b]) - r))
        fs.append(abs(r - float(v[i, j, b])))
    print(f"  max err {max(errs):.2e}, max |f| {max(fs):.2e}", flush=True)
    assert max(errs) <= 2e-3 * max(fs) + 1e-6


@pytest.mark.parametrize("shape", [(2, 7, 9, 21), (1, 1, 5, 3), (3, 5, 4, 17)])
def test_forward_and_gradient_within_storage_bound_of_exact_network(device, shape):
    """u0, the loss and every parameter block of the gradient against the exact FP64 network,
    within LAMBDA x the spread of bfloat16-sized storage errors (per output block)."""
    import cnn_error_bound as eb
    print(f"exact-network bound shape={shape}", flush=True)
    v, target = _inputs(shape, 81)
    params = synth.cnn_random_params(seed=82)
    p64, v64, t64 = params.astype(np.float64), v.astype(np.float64), target.astype(np.float64)
    tp, tv = torch.from_numpy(params).to(device), torch.from_numpy(v).to(device)
    u0 = nt.cnn_forward(tp, tv).cpu().numpy().astype(np.float64)
    ref, spread = eb.forward_spread(p64, v64)
    r = np.linalg.norm(u0 - ref) / spread
    print(f"  u0: error / spread {r:.2f}", flush=True)
    assert r <= eb.LAMBDA
    loss, grad = nt.cnn_grad(tp, tv, torch.from_numpy(target).to(device))
    g = grad.cpu().numpy().astype(np.float64)
    rl, rg, sp, sp_loss = eb.grad_spread(p64, v64, t64)
    print(f"  loss: error / spread {abs(loss - rl) / sp_loss:.2f}", flush=True)
    assert abs(loss - rl) <= eb.LAMBDA * sp_loss + 1e-6 * abs(rl)
    for name, a, b in eb.blocks():
        r = np.linalg.norm(g[a:b] - rg[a:b]) / sp[name]
        print(f"  {name}: error / spread {r:.2f}", flush=True)
        assert r <= eb.LAMBDA, name
