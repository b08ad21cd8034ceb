"""Batched solve (s3ttv_solve_batched): every problem's result is identical to its standalone
s3ttv_solve, across shapes that take each block-pass route, graph replays, per-problem stop
rules and budgets, and a failing problem next to healthy ones."""
import numpy as np
import pytest

from paper_2404_03313_amd import native as nt
from paper_2404_03313_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _t(x, device):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(device)


def _np(x):
    return x.detach().cpu().numpy()


def _problem(device, shape, k, seed, **kw):
    cfg = synth.HSIConfig(*shape, endmembers=3, cells=5, sigma=0.08, p_sp=0.05, p_stripe=0.2,
                          seed=seed)
    d = synth.make_hsi(cfg)
    prm = nt.make_params(**d["radii"], **kw)
    return dict(v=_t(d["v"], device), k1=k[0], k2=k[1], params=prm)


# fused pass (k 3x3, 2x3; 20 column tiles at N3 = 150), separate kernels (N3 > 192), separate
# overlap-add sum (ragged tiles)
SHAPES = [((24, 20, 16), (3, 3)), ((13, 11, 7), (2, 3)), ((12, 10, 150), (2, 2)),
          ((12, 10, 200), (2, 2)), ((10, 10, 8), (4, 4))]


def _standalone(p):
    prm = p["params"]
    n1, n2, n3 = p["v"].shape
    sv = nt.Solver(n1, n2, n3, p["k1"], p["k2"], device=p["v"].device)
    return sv.solve(p["v"], prm, u0=p.get("u0"))


def _same(batched, single, label):
    for name, a, b in zip("ust", batched[:3], single[:3]):
        assert np.array_equal(_np(a), _np(b)), (label, name, np.abs(_np(a) - _np(b)).max())
    assert batched[3]["iters"] == single[3]["iters"], label
    assert batched[3]["converged"] == single[3]["converged"], label


def test_batched_matches_standalone_fixed_iterations(device):
    """40 iterations: the first directly, two replays of the 16-iteration graph, a direct tail."""
    _say("batched: 4 shapes x 40 iterations")
    probs = [_problem(device, sh, k, 20 + i, max_iter=40) for i, (sh, k) in enumerate(SHAPES)]
    res, rc = nt.solve_batched(probs)
    assert rc == nt.OK
    for i, p in enumerate(probs):
        _say("  problem", i, "tile", res[i][3]["tile"], "iters", res[i][3]["iters"])
        _same(res[i], _standalone(p), i)


def test_batched_stop_rules_and_budgets(device):
    """Problems stop on their own rule or budget; a problem whose budget runs out before its
    rule fires reports NOT_CONVERGED, the call as a whole too."""
    _say("batched: stop rules")
    probs = [_problem(device, SHAPES[0][0], SHAPES[0][1], 31, max_iter=3000, rel_tol=2e-3),
             _problem(device, SHAPES[1][0], SHAPES[1][1], 32, max_iter=70),
             _problem(device, SHAPES[3][0], SHAPES[3][1], 33, max_iter=25, rel_tol=1e-9)]
    res, rc = nt.solve_batched(probs)
    assert rc == nt.NOT_CONVERGED
    assert res[0][3]["converged"] and res[0][3]["status"] == nt.OK
    assert res[1][3]["iters"] == 70 and res[1][3]["status"] == nt.OK
    assert res[2][3]["iters"] == 25 and res[2][3]["status"] == nt.NOT_CONVERGED
    for i, p in enumerate(probs):
        _say("  problem", i, "iters", res[i][3]["iters"], "converged", res[i][3]["converged"])
        _same(res[i], _standalone(p), i)


def test_batched_failing_problem_is_isolated(device):
    _say("batched: non-finite input in one problem")
    probs = [_problem(device, sh, k, 40 + i, max_iter=20) for i, (sh, k) in enumerate(SHAPES[:2])]
    bad = probs[1]["v"].clone()
    bad[0, 0, 0] = float("nan")
    probs[1]["v"] = bad
    with pytest.raises(nt.S3TTVError) as e:
        nt.solve_batched(probs)
    assert e.value.code == nt.ENONFINITE


def test_batched_repeated_calls_are_identical(device):
    """The captured graph is rebuilt per call; two calls (second with a smaller batch) agree."""
    _say("batched: repeated calls")
    probs = [_problem(device, sh, k, 50 + i, max_iter=35) for i, (sh, k) in enumerate(SHAPES)]
    res1, _ = nt.solve_batched(probs)
    res2, _ = nt.solve_batched(probs[:2])
    for i in range(2):
        for a, b in zip(res1[i][:3], res2[i][:3]):
            assert np.array_equal(_np(a), _np(b)), i
