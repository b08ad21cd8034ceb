"""Operator-level parity of the HIP kernels (through the C ABI) against the FP64 oracle.

Each case prints its name and shape before the GPU call. Tolerances follow from FP32
arithmetic on inputs of magnitude <= ~1 (see the design notes): stencils and block steps
agree to ~1e-6 relative, the l1 threshold to ~1e-12 relative (exact-sum selection in
FP64 on both sides).
"""
import os

import numpy as np
import pytest

import oracle
from paper_2404_03313_amd import native as nt

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _t(x, device):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(device)


def _np(x):
    return x.detach().cpu().numpy().astype(np.float64)


GRAD_SHAPES = [(32, 32, 16), (13, 11, 7), (2, 3, 2), (9, 20, 33), (64, 48, 128)]


@pytest.mark.parametrize("shape", GRAD_SHAPES)
def test_grad_matches_oracle(device, shape):
    _say("op_grad", shape)
    rng = np.random.default_rng(1)
    u32 = rng.uniform(0, 1, size=shape).astype(np.float32)
    u = u32.astype(np.float64)
    gv, gh = nt.op_grad(_t(u32, device))
    ds = oracle.ds(u)
    np.testing.assert_allclose(_np(gv), oracle.dv(ds), atol=2e-6, rtol=0)
    np.testing.assert_allclose(_np(gh), oracle.dh(ds), atol=2e-6, rtol=0)


@pytest.mark.parametrize("shape", GRAD_SHAPES)
def test_grad_adjoint_matches_oracle(device, shape):
    _say("op_grad_adj", shape)
    rng = np.random.default_rng(2)
    zv32 = rng.normal(size=shape).astype(np.float32)
    zh32 = rng.normal(size=shape).astype(np.float32)
    w = nt.op_grad_adj(_t(zv32, device), _t(zh32, device))
    want = oracle.ds_t(oracle.dv_t(zv32.astype(np.float64)) + oracle.dh_t(zh32.astype(np.float64)))
    np.testing.assert_allclose(_np(w), want, atol=1e-5, rtol=0)


CLIP_CASES = [(37, 16, 256), (64, 9, 32), (5, 16, 8), (130, 4, 382), (3, 1, 17), (70, 16, 48)]


@pytest.mark.parametrize("nblk,K,ncols", CLIP_CASES)
def test_spectral_clip_matches_oracle(device, nblk, K, ncols):
    _say("op_spectral_clip", nblk, K, ncols)
    rng = np.random.default_rng(3)
    Y = rng.normal(size=(nblk, K, ncols))
    # spread spectral norms around 1 so both branches of the clip are exercised
    scale = rng.uniform(0.3, 3.0, size=(nblk, 1, 1)) / np.sqrt(ncols)
    Y32 = (Y * scale).astype(np.float32)
    got = _np(nt.op_spectral_clip(_t(Y32, device)))
    Y64 = Y32.astype(np.float64)
    for b in range(nblk):
        want = oracle.dual_nuclear(Y64[b], 0.25)
        err = np.linalg.norm(got[b] - want) / max(np.linalg.norm(want), 1e-30)
        assert err < 2e-5, (b, err)
        assert np.linalg.norm(got[b], 2) <= 1 + 1e-4


def test_spectral_clip_special_cases(device):
    _say("op_spectral_clip special")
    K, ncols = 16, 64
    Ys = []
    Ys.append(np.zeros((K, ncols)))                              # zero block
    a = np.linalg.qr(np.random.default_rng(4).normal(size=(K, K)))[0][:, 0]
    bvec = np.random.default_rng(5).normal(size=ncols); bvec /= np.linalg.norm(bvec)
    Ys.append(3.0 * np.outer(a, bvec))                           # rank 1, sigma 3 -> 1
    Ys.append(0.5 * np.outer(a, bvec))                           # inside the ball: unchanged
    D = np.zeros((K, ncols)); D[np.arange(K), np.arange(K)] = np.linspace(-2, 2, K)
    Ys.append(D)                                                 # diagonal: clip entries
    Y32 = np.stack(Ys).astype(np.float32)
    got = _np(nt.op_spectral_clip(_t(Y32, device)))
    np.testing.assert_array_equal(got[0], 0)
    np.testing.assert_allclose(got[1], np.outer(a, bvec), atol=2e-6)
    np.testing.assert_allclose(got[2], Y32[2].astype(np.float64), atol=1e-7)
    want = np.zeros((K, ncols))
    d = np.linspace(-2, 2, K).astype(np.float32).astype(np.float64)
    want[np.arange(K), np.arange(K)] = np.sign(d) * np.minimum(np.abs(d), 1)
    np.testing.assert_allclose(got[3], want, atol=2e-6)


DUAL_CASES = [((32, 32, 16), (3, 3)), ((13, 11, 7), (2, 3)), ((9, 20, 33), (4, 4)),
              ((4, 6, 5), (4, 4)), ((2, 3, 2), (2, 3)), ((17, 9, 16), (1, 1)), ((24, 40, 20), (4, 2)),
              # more than 16 rows: the one-workgroup-per-block kernel (K = 20, 21, 100; the last
              # window covers the whole 10 x 10 image, and K exceeds the 2 N3 = 40 columns)
              ((12, 11, 9), (5, 4)), ((7, 13, 33), (3, 7)), ((10, 10, 20), (10, 10)),
              # overlap-add accumulators of 11 x 11 pixels x 144 columns: more than 64 KB of LDS
              ((24, 24, 64), (4, 4))]


@pytest.mark.parametrize("shape,k", DUAL_CASES)
def test_dual_blocks_match_oracle(device, shape, k):
    """Alg. 1 steps 9-10 on every block plus the overlap-add (P^T) of the result."""
    k1, k2 = k
    _say("op_dual_blocks", shape, k)
    rng = np.random.default_rng(6)
    n1, n2, n3 = shape
    up32 = rng.uniform(-0.5, 1.5, size=shape).astype(np.float32)
    Y32 = (rng.normal(size=(n1 * n2, k1 * k2, 2 * n3)) * 0.3 / np.sqrt(2 * n3)).astype(np.float32)
    yout, zv, zh = nt.op_dual_blocks(_t(up32, device), _t(Y32, device), k1, k2, 0.25)
    T = oracle.struct_tensor(up32.astype(np.float64), k1, k2)
    Yp = Y32.astype(np.float64) + 0.25 * T
    want = np.stack([oracle.dual_nuclear(Yp[l], 0.25) for l in range(n1 * n2)])
    got = _np(yout)
    scale = max(np.abs(want).max(), 1e-6)
    assert np.abs(got - want).max() < 3e-5 * scale
    wzv, wzh = oracle.blocks_scatter(want, shape, k1, k2)
    zs = max(np.abs(wzv).max(), np.abs(wzh).max())
    assert np.abs(_np(zv) - wzv).max() < 1e-4 * zs
    assert np.abs(_np(zh) - wzh).max() < 1e-4 * zs


@pytest.mark.parametrize("k", [(4, 4), (5, 4)])
def test_dual_blocks_nonfinite_input(device, k):
    """A NaN in one block is reported as ENONFINITE by both block routes (16 rows or fewer,
    and more)."""
    _say("op_dual_blocks NaN", k)
    rng = np.random.default_rng(8)
    n1, n2, n3 = 9, 8, 6
    up = rng.uniform(0, 1, size=(n1, n2, n3)).astype(np.float32)
    Y = (rng.normal(size=(n1 * n2, k[0] * k[1], 2 * n3)) * 0.05).astype(np.float32)
    Y[5, 3, 7] = np.nan
    with pytest.raises(nt.S3TTVError) as ei:
        nt.op_dual_blocks(_t(up, device), _t(Y, device), k[0], k[1], 0.25)
    assert ei.value.code == nt.ENONFINITE


def test_dual_blocks_first_call_in_process(device):
    """The operator raises the block kernels' LDS limit itself: called first in a fresh
    process at a shape whose overlap-add needs more than 64 KB of LDS, it still runs."""
    import subprocess
    import sys
    _say("op_dual_blocks first call in a fresh process")
    code = (
        "import numpy as np, torch\n"
        "from paper_2404_03313_amd import native as nt\n"
        "rng = np.random.default_rng(3)\n"
        "up = torch.from_numpy(rng.uniform(0, 1, size=(24, 24, 64)).astype(np.float32)).cuda()\n"
        "Y = torch.zeros(24 * 24, 16, 128, device='cuda')\n"
        "yout, zv, zh = nt.op_dual_blocks(up, Y, 4, 4, 0.25)\n"
        "torch.cuda.synchronize()\n"
        "assert bool(torch.isfinite(yout).all()) and float(yout.abs().max()) > 0\n"
        "print('ok')\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().endswith("ok")


L1_CASES = ["normal_large", "ties", "inside", "single", "zeros_denormals", "spiky", "c2_size",
            "one_bin", "misaligned"]


@pytest.mark.parametrize("case", L1_CASES)
def test_l1_projection_matches_oracle(device, case):
    _say("op_l1_project", case)
    rng = np.random.default_rng(7)
    if case == "normal_large":
        x = rng.normal(size=1_000_003) * 0.2
        r = 0.3 * np.abs(x).sum()
    elif case == "ties":
        x = np.repeat(rng.normal(size=50), 997) * 0.5
        r = 0.1 * np.abs(x).sum()
    elif case == "inside":
        x = rng.normal(size=4097)
        r = 2 * np.abs(x).sum()
    elif case == "single":
        x = np.array([-3.0])
        r = 1.25
    elif case == "zeros_denormals":
        x = np.concatenate([np.zeros(1000), np.full(100, 1e-40), rng.normal(size=5000) * 1e-3])
        r = 0.5 * np.abs(x.astype(np.float32)).sum()
    elif case == "spiky":
        x = rng.normal(size=200000) * 1e-3
        x[rng.choice(x.size, 300, replace=False)] = rng.choice([-1, 1], 300) * rng.uniform(0.5, 5, 300)
        r = 0.7 * np.abs(x).sum()
    elif case == "misaligned":
        # passed as a view 4 bytes into its allocation (no 16-byte alignment)
        x = rng.normal(size=300_001) * 0.3
        r = 0.2 * np.abs(x).sum()
    elif case == "one_bin":
        # every |x| in [0.5, 0.55): one level-1 bin, so levels 2-3 see all elements
        x = 0.5 * (1 + 0.1 * rng.uniform(size=1 << 20)) * rng.choice([-1, 1], 1 << 20)
        r = 0.3 * np.abs(x).sum()
    else:
        x = rng.normal(size=256 * 256 * 128) * 0.05
        x[rng.choice(x.size, 400000, replace=False)] += rng.choice([-0.7, 0.7], 400000)
        r = 0.95 * 0.05 * x.size / 2
    x32 = x.astype(np.float32)
    if case == "misaligned":
        buf = _t(np.concatenate([[0.0], x32]), device)
        xin = buf[1:]
        assert xin.data_ptr() % 16 != 0
    else:
        xin = _t(x32, device)
    got, tau = nt.op_l1_project(xin, r)
    want, wtau = oracle.proj_l1(x32.astype(np.float64), r)
    if wtau == 0:
        assert tau == 0
    else:
        assert abs(tau - wtau) <= 1e-12 * wtau + 1e-300, (tau, wtau)
    np.testing.assert_allclose(_np(got), want, atol=2e-7 * max(np.abs(x32).max(), 1e-30), rtol=0)
