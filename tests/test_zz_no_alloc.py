"""s3ttv_op_l1_project_noalloc (the l1-ball projection with the library's static scratch
instead of a workspace) against s3ttv_op_l1_project on the same inputs: two calls in a row,
the second on a smaller input, so that what the first call left in the shared scratch must not
change the second result. Same kernels, so the outputs and thresholds must agree bitwise."""
import numpy as np
import pytest
import torch

from paper_2404_03313_amd import native as nt

pytestmark = pytest.mark.gpu


def _x(n, seed, device):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.normal(0, 1, n) * rng.uniform(0, 1, n) ** 3   # heavy-tailed magnitudes, mixed signs
    x[rng.integers(0, n, max(n // 50, 1))] = 0.0
    return torch.from_numpy(x.astype(np.float32)).to(device)


def test_noalloc_matches_workspace_entry_point(device):
    for n, seed, frac in ((3_000_001, 1, 0.3), (40_001, 2, 0.5), (7, 3, 0.2)):
        print(f"noalloc l1 projection n={n} seed={seed}", flush=True)
        x = _x(n, seed, device)
        radius = frac * float(x.abs().double().sum())
        ref, tau_ref = nt.op_l1_project(x, radius)
        got, tau = nt.op_l1_project_noalloc(x, radius)
        assert tau_ref > 0.0
        assert tau == tau_ref
        assert torch.equal(got, ref)
        assert float(got.abs().double().sum()) <= radius * (1 + 1e-6)
    # inside the ball: the identity, threshold 0
    x = _x(1000, 4, device)
    got, tau = nt.op_l1_project_noalloc(x, 2.0 * float(x.abs().double().sum()))
    assert tau == 0.0 and torch.equal(got, x)


def test_noalloc_rejects_more_than_its_scratch_holds(device):
    x = torch.zeros((1 << 24) + 1, device=device)
    with pytest.raises(nt.S3TTVError) as e:
        nt.op_l1_project_noalloc(x, 1.0)
    assert e.value.code == nt.EUNSUPPORTED
    out, tau = nt.op_l1_project_noalloc(x[: 1 << 24], 1.0)   # the largest size it takes
    assert tau == 0.0 and torch.equal(out, x[: 1 << 24])
