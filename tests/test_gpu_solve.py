"""End-to-end parity of the GPU solver (s3ttv_solve through the C ABI) with the FP64 oracle.

The bar is a relative L2 error <= 1e-4 per output (u, s, t) after a fixed iteration count,
FP32 GPU against FP64 oracle on the same float32 observation. Invariants that hold at any
size are checked at the full 256 x 256 x 128 throughput shape.
"""
import numpy as np
import pytest

import oracle
from paper_2404_03313_amd import native as nt
from paper_2404_03313_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _t(x, device):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(device)


def _np(x):
    return x.detach().cpu().numpy().astype(np.float64)


def rel_l2(a, b):
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-12 * np.sqrt(b.size))


def _parity(device, d, k, iters, tol=1e-4, **kw):
    k1, k2 = k
    v = d["v"]
    u, s, t, st = nt.solve(_t(v, device), k1, k2, max_iter=iters, **d["radii"], **kw)
    kw_o = {key: val for key, val in kw.items() if key in ("rel_tol", "gammas")}
    for key in ("u0", "s0", "t0"):
        if key in kw:
            kw_o[key] = _np(kw[key])
    r = oracle.solve(d["v64"], k1, k2, max_iter=iters, **d["radii"], **kw_o)
    errs = {name: rel_l2(_np(g), r[name]) for name, g in (("u", u), ("s", s), ("t", t))}
    _say("rel L2 vs oracle:", errs, "gpu iters", st["iters"], "oracle iters", r["stats"]["iters"],
         "max sweeps", st["eig_max_sweeps"], "avg steps", st["eig_avg_steps"],
         "fallback blocks", st["eig_fallback_blocks"])
    for name, e in errs.items():
        assert e <= tol, (name, e)
    return u, s, t, st, r


def test_solve_parity_small_workload(device):
    """32 x 32 x 16, block 3 x 3, 200 iterations (the parity workload)."""
    _say("solve c1 200 iters")
    w = synth.WORKLOADS["c1"]
    d = synth.make_hsi(w["cfg"])
    u, s, t, st, r = _parity(device, d, w["k"], w["iters"])
    assert st["iters"] == 200
    un = _np(u)
    assert un.min() >= 0.0 and un.max() <= 1.0
    assert st["l1_s"] <= d["radii"]["alpha"] * (1 + 1e-5)
    assert st["l1_t"] <= d["radii"]["beta"] * (1 + 1e-5)


@pytest.mark.parametrize("shape,k,iters", [((13, 11, 7), (2, 3), 60), ((20, 24, 33), (4, 4), 40),
                                           ((6, 5, 3), (1, 2), 80), ((16, 16, 16), (4, 1), 50),
                                           # ragged wrapping tiles: more than 4 overlap-add
                                           # partials per pixel, summed by the separate pass
                                           ((10, 10, 8), (4, 4), 40),
                                           # four-band primal path: one quad per pixel (every
                                           # lane gathers the band below), and three per pixel
                                           # with pixels split across wavefronts and a partial
                                           # last wavefront
                                           ((12, 9, 4), (2, 2), 60), ((11, 13, 12), (3, 3), 40)])
def test_solve_parity_ragged(device, shape, k, iters):
    _say("solve ragged", shape, k, iters)
    cfg = synth.HSIConfig(*shape, endmembers=3, cells=5, sigma=0.08, p_sp=0.05, p_stripe=0.2, seed=11)
    d = synth.make_hsi(cfg)
    _parity(device, d, k, iters)


def test_solve_parity_custom_steps_and_warm_start(device):
    _say("solve custom gammas + u0")
    cfg = synth.HSIConfig(16, 12, 10, endmembers=3, cells=4, sigma=0.05, p_sp=0.05, p_stripe=0.2, seed=12)
    d = synth.make_hsi(cfg)
    g = dict(nt.default_gammas(2, 2))
    g["gamma_u"] = 1.0 / (8 * 16 * 4 + 1)   # the printed (more conservative) value of eq. stepsize_denoising
    u0 = _t(np.clip(d["v"], 0, 1), device)
    _parity(device, d, (2, 2), 40, gammas=g, u0=u0)


def test_solve_from_primal_starts(device):
    """s3ttv_solve_from: u0, s0 and t0 all given (Alg. 1 leaves every initial value free)."""
    _say("solve from u0, s0, t0")
    cfg = synth.HSIConfig(14, 12, 9, endmembers=3, cells=4, sigma=0.05, p_sp=0.05, p_stripe=0.2, seed=13)
    d = synth.make_hsi(cfg)
    rng = np.random.Generator(np.random.PCG64(14))
    v = d["v"].astype(np.float64)
    u0 = np.clip(v, 0, 1)
    r = v - u0 + rng.normal(0, 0.05, size=v.shape)
    s0 = np.where(np.abs(r) > 0.1, r, 0.0)
    t0 = np.broadcast_to(rng.uniform(-0.2, 0.2, size=(1,) + v.shape[1:]), v.shape)
    _parity(device, d, (2, 2), 50, u0=_t(u0, device), s0=_t(s0, device), t0=_t(t0, device))
    bad = s0.copy()
    bad[3, 4, 5] = np.nan
    with pytest.raises(nt.S3TTVError) as e:
        nt.solve(_t(d["v"], device), 2, 2, max_iter=5, **d["radii"], s0=_t(bad, device))
    assert e.value.code == nt.ENONFINITE


@pytest.mark.parametrize("steps", [-1, 1])
def test_solve_parity_eigen_fallback(device, steps):
    """Few (or no) MFMA rotation steps: most blocks go through the per-lane Jacobi and the
    fix-up of the fused block pass; the result must not change beyond rounding."""
    _say("solve c1 eig_max_steps", steps)
    w = synth.WORKLOADS["c1"]
    d = synth.make_hsi(w["cfg"])
    u, s, t, st, r = _parity(device, d, w["k"], 60, eig_max_steps=steps)
    assert st["eig_fallback_blocks"] > 0


@pytest.mark.parametrize("prec,tol", [(nt.GRAM_BF16, 1e-5), (nt.GRAM_FP16, 5e-6)])
def test_solve_parity_reduced_precision_gram(device, prec, tol):
    """Block Gram products with BF16 / FP16 inputs (FP32 accumulation), the eigenvectors then
    refined by one FP32 step against the Gram corrected by the inputs' rounding residual,
    everything else FP32, against the FP64 oracle on the parity workload. Measured on MI355X:
    BF16 up to 1.4e-6, FP16 up to 8.0e-7 relative L2 (t the largest; FP32 itself 8.2e-7).
    Without the refinement step they were 6.4e-5 and 6.5e-6."""
    _say("solve c1 gram precision", prec)
    w = synth.WORKLOADS["c1"]
    d = synth.make_hsi(w["cfg"])
    _parity(device, d, w["k"], w["iters"], tol=tol, gram_precision=prec)


@pytest.mark.parametrize("n3,route", [(150, "block"), (180, "block"), (200, "gram")])
def test_solve_parity_many_bands(device, n3, route):
    """Many bands: up to 24 column tiles (N3 <= 192) the fused pass (an 8 x 4 anchor tile, the
    accumulators of 8 x 8 no longer fit the LDS), beyond it the separate Gram / eigen / apply
    kernels."""
    _say(f"solve 12x10x{n3}")
    cfg = synth.HSIConfig(12, 10, n3, endmembers=3, cells=4, sigma=0.05, p_sp=0.05, p_stripe=0.2, seed=14)
    d = synth.make_hsi(cfg)
    u, s, t, st, r = _parity(device, d, (2, 2), 40)
    assert st["eig_avg_steps"] > 0
    # the route shows in which kernels run (a timed solve counts their launches)
    prm = nt.make_params(max_iter=3, timing_mask=(1 << nt.K_BLOCK) | (1 << nt.K_GRAM), **d["radii"])
    _, _, _, st3 = nt.Solver(12, 10, n3, 2, 2, device=device).solve(_t(d["v"], device), prm)
    assert st3["kernel_calls"][route] == 3, st3["kernel_calls"]
    other = "gram" if route == "block" else "block"
    assert st3["kernel_calls"][other] == 0, st3["kernel_calls"]


def test_solve_stop_rule_matches_oracle(device):
    _say("solve rel_tol")
    cfg = synth.HSIConfig(12, 12, 8, endmembers=3, cells=4, sigma=0.05, p_sp=0.05, p_stripe=0.2, seed=13)
    d = synth.make_hsi(cfg)
    u, s, t, st, r = _parity(device, d, (2, 2), 2000, rel_tol=2e-3, check_every=7)
    assert st["converged"] and r["stats"]["converged"]
    assert abs(st["iters"] - r["stats"]["iters"]) <= 1


def test_stop_rule_value_matches_separate_oracle_runs(device):
    """The relative change the GPU reports after k iterations (the quantity of eq.
    StopCri_simulated) equals ||u^(k) - u^(k-1)|| / ||u^(k-1)|| formed from two oracle runs of
    k - 1 and k iterations."""
    _say("solve stop-rule value")
    cfg = synth.HSIConfig(12, 12, 8, endmembers=3, cells=4, sigma=0.05, p_sp=0.05, p_stripe=0.2, seed=13)
    d = synth.make_hsi(cfg)
    v = _t(d["v"], device)
    for k in (3, 5, 9, 40):
        st = nt.solve(v, 2, 2, max_iter=k, **d["radii"])[3]
        prev = oracle.solve(d["v64"], 2, 2, max_iter=k - 1, **d["radii"])["u"]
        cur = oracle.solve(d["v64"], 2, 2, max_iter=k, **d["radii"])["u"]
        want = np.linalg.norm(cur - prev) / np.linalg.norm(prev)
        _say("  k", k, "gpu", st["rel_change"], "from oracle runs", want)
        assert st["rel_change"] == pytest.approx(want, rel=1e-4)


def test_solve_deterministic(device):
    _say("solve determinism")
    d = synth.make_hsi(synth.WORKLOADS["c1"]["cfg"])
    a = nt.solve(_t(d["v"], device), 3, 3, max_iter=30, **d["radii"])
    b = nt.solve(_t(d["v"], device), 3, 3, max_iter=30, **d["radii"])
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(_np(x), _np(y))


def test_solve_errors(device):
    import torch
    _say("solve error codes")
    v = torch.zeros((8, 8, 4), device=device)
    v[1, 2, 3] = float("nan")
    with pytest.raises(nt.S3TTVError) as e:
        nt.solve(v, 2, 2, 1.0, 1.0, 1.0, 5)
    assert e.value.code == nt.ENONFINITE
    with pytest.raises(nt.S3TTVError) as e:   # blocks of more than 100 rows
        nt.solve(torch.zeros((12, 12, 4), device=device), 11, 10, 1.0, 1.0, 1.0, 5)
    assert e.value.code == nt.EUNSUPPORTED


@pytest.mark.timeout(900)
def test_large_shape_first_iterations_and_invariants(device):
    """256 x 256 x 128, block 4 x 4: elementwise parity after 3 iterations, then feasibility
    invariants after 100 iterations (box, both l1 balls), in the benchmark's configuration."""
    _say("solve 256x256x128: 3 iterations vs oracle")
    w = synth.WORKLOADS["c2"]
    d = synth.make_hsi(w["cfg"])
    k1, k2 = w["k"]
    v = _t(d["v"], device)
    u, s, t, st = nt.solve(v, k1, k2, max_iter=3, **d["radii"])
    r = oracle.solve(d["v64"], k1, k2, max_iter=3, **d["radii"])
    for name, g in (("u", u), ("s", s), ("t", t)):
        e = rel_l2(_np(g), r[name])
        _say(name, "rel L2", e)
        assert e <= 1e-5
    _say("solve 256x256x128: 100 iterations, invariants")
    u, s, t, st = nt.solve(v, k1, k2, max_iter=100, **d["radii"])
    un = _np(u)
    assert un.min() >= 0.0 and un.max() <= 1.0
    assert st["l1_s"] <= d["radii"]["alpha"] * (1 + 1e-5)
    assert st["l1_t"] <= d["radii"]["beta"] * (1 + 1e-5)
    assert np.isfinite(st["fid"]) and np.isfinite(st["dv_t"])
    _say("stats", {k: st[k] for k in ("iters", "fid", "dv_t", "eig_max_sweeps", "eig_avg_steps",
                                      "eig_max_steps", "eig_fallback_blocks", "ms")})


@pytest.mark.parametrize("shape,k,reg", [((32, 32, 16), (3, 3), "s3ttv"), ((12, 12, 8), (10, 10), "s3ttv"),
                                         ((20, 16, 12), (2, 2), "sstv")])
def test_graph_replay_matches_direct_launches(device, shape, k, reg):
    """The solve replays one captured graph of iterations (after the first) unless kernel
    timing is requested, which launches every kernel directly. Both must give bitwise the same
    result and iteration count: a fixed budget (first iteration, three replays, a direct
    remainder) and a stop rule that fires inside a replay; two graph solves in a row with
    other work between them agree too."""
    import torch
    _say("graph replay vs direct launches", shape, k, reg)
    cfg = synth.HSIConfig(*shape, endmembers=3, cells=5, sigma=0.08, p_sp=0.05, p_stripe=0.2,
                          seed=77)
    d = synth.make_hsi(cfg)
    v = _t(d["v"], device)
    sv = nt.Solver(*shape, *k, device=device)
    for kw in (dict(max_iter=61), dict(max_iter=5000, rel_tol=1e-4)):
        g = sv.solve(v, nt.make_params(regularizer=reg, **kw, **d["radii"]))
        g = tuple(x.clone() for x in g[:3]) + (g[3],)
        torch.ones(1 << 20, device=device).sum().item()   # eager work between the solves
        g2 = sv.solve(v, nt.make_params(regularizer=reg, **kw, **d["radii"]))
        dl = sv.solve(v, nt.make_params(regularizer=reg, timing_mask=1 << nt.K_FINAL, **kw,
                                        **d["radii"]))
        for a, b, c in zip(g[:3], g2[:3], dl[:3]):
            assert torch.equal(a, b) and torch.equal(a, c)
        assert g[3]["iters"] == g2[3]["iters"] == dl[3]["iters"]
        _say("  ", kw, "iterations", g[3]["iters"])


@pytest.mark.parametrize("shape,k,reg", [((32, 32, 16), (3, 3), "s3ttv"), ((12, 10, 150), (2, 2), "s3ttv"),
                                         ((12, 12, 8), (10, 10), "s3ttv"), ((20, 16, 12), (2, 2), "sstv"),
                                         ((14, 13, 9), (3, 2), "stv")])
def test_continue_equals_one_uninterrupted_solve(device, shape, k, reg):
    """s3ttv_solve_continue: a solve of n1 iterations continued by n2 gives bitwise the solve of
    n1 + n2 iterations (graph replays and direct launches, every block-pass route, an l1
    variant); a continued stop rule fires at the iteration of the uninterrupted solve."""
    import torch
    _say("continue", shape, k, reg)
    cfg = synth.HSIConfig(*shape, endmembers=3, cells=5, sigma=0.08, p_sp=0.05, p_stripe=0.2,
                          seed=91)
    d = synth.make_hsi(cfg)
    v = _t(d["v"], device)
    sv = nt.Solver(*shape, *k, device=device)
    ref = sv.solve(v, nt.make_params(max_iter=57, regularizer=reg, **d["radii"]))
    ref = tuple(x.clone() for x in ref[:3])
    for n1, timing in ((20, 0), (1, 0), (36, 1 << nt.K_FINAL)):
        sv.solve(v, nt.make_params(max_iter=n1, regularizer=reg, **d["radii"]))
        got = sv.resume(v, nt.make_params(max_iter=57 - n1, regularizer=reg, timing_mask=timing,
                                          **d["radii"]))
        assert got[3]["iters"] == 57 - n1
        for a, b in zip(got[:3], ref):
            assert torch.equal(a, b), (n1, timing)
    # continued in three pieces
    sv.solve(v, nt.make_params(max_iter=10, regularizer=reg, **d["radii"]))
    sv.resume(v, nt.make_params(max_iter=30, regularizer=reg, **d["radii"]))
    got = sv.resume(v, nt.make_params(max_iter=17, regularizer=reg, **d["radii"]))
    for a, b in zip(got[:3], ref):
        assert torch.equal(a, b)
    # the stop rule in a continuation
    one = sv.solve(v, nt.make_params(max_iter=5000, rel_tol=1e-3, regularizer=reg, **d["radii"]))
    n_one = one[3]["iters"]
    one = tuple(x.clone() for x in one[:3])
    sv.solve(v, nt.make_params(max_iter=7, regularizer=reg, **d["radii"]))
    got = sv.resume(v, nt.make_params(max_iter=5000, rel_tol=1e-3, regularizer=reg, **d["radii"]))
    _say("  stop rule after", n_one, "iterations; continued", 7, "+", got[3]["iters"])
    assert got[3]["converged"] and got[3]["iters"] == n_one - 7
    for a, b in zip(got[:3], one):
        assert torch.equal(a, b)


def test_continue_rejects_a_workspace_without_that_state(device):
    import torch
    _say("continue errors")
    d = synth.make_hsi(synth.HSIConfig(12, 12, 8, endmembers=3, cells=4, sigma=0.05, p_sp=0.05,
                                       p_stripe=0.2, seed=13))
    v = _t(d["v"], device)
    sv = nt.Solver(12, 12, 8, 2, 2, device=device)
    sv.ws.zero_()
    with pytest.raises(nt.S3TTVError) as e:      # never solved
        sv.resume(v, nt.make_params(max_iter=5, **d["radii"]))
    assert e.value.code == nt.EINVAL
    sv.solve(v, nt.make_params(max_iter=5, regularizer="sstv", **d["radii"]))
    with pytest.raises(nt.S3TTVError) as e:      # another regulariser
        sv.resume(v, nt.make_params(max_iter=5, **d["radii"]))
    assert e.value.code == nt.EINVAL
    sv.solve(v, nt.make_params(max_iter=5, **d["radii"]))
    other = nt.Solver(12, 12, 8, 2, 2, device=device)
    other.ws.copy_(sv.ws)
    other.shape = nt.Shape(12, 12, 8, 1, 2)       # another block size on the same bytes
    with pytest.raises(nt.S3TTVError) as e:
        other.resume(v, nt.make_params(max_iter=5, **d["radii"]))
    assert e.value.code == nt.EINVAL
    torch.cuda.synchronize()
