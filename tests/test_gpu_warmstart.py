"""What the learned initial estimate gains (GPU). The network is trained by the library's
own kernels on solver-generated pairs; held-out scenes are then solved from u0 = 0 and from
u0 = v + f(v). Prob. (18) is convex with (measured) a unique solution, so every start ends at
the same point: the zero-start run is the yardstick for the warm-started one.

What is asserted is what holds scene after scene: the estimate is far closer to the solution
than the observation; the iterates stay closer to the solution during the first hundred
iterations; the paper's stop rule (relative change below 1e-4) is met in fewer iterations in
total; and long runs from both starts meet. The duals still start at zero, so the warm run
does not converge faster to tight tolerances (documented with measurements, not asserted).
"""
import numpy as np
import pytest
import torch

from paper_2404_03313_amd import native as nt
from paper_2404_03313_amd import synth
from paper_2404_03313_amd import warmstart as ws

pytestmark = pytest.mark.gpu


def _dist(a, b):
    return float((a - b).norm() / b.norm())


@pytest.fixture(scope="module")
def trained(device):
    print("pairs: 64 scenes 64^3", flush=True)
    V, U, _ = ws.make_pairs(synth.cnn_train_configs(count=64), rel_tol=1e-5, max_iter=3000,
                            device=device)
    tr = ws.Trainer(synth.cnn_init(0), device=device)
    before = tr.loss(V, U)
    losses = tr.train(V, U, steps=300, batch=8, lr=1e-3)
    after = tr.loss(V, U)
    print(f"training loss {before:.3e} -> {after:.3e}", flush=True)
    del V, U
    return tr, before, after, losses


def test_training_reduces_the_loss(trained):
    _, before, after, losses = trained
    assert np.isfinite(losses).all()
    assert after < 0.2 * before


def test_trained_network_gains_on_held_out_scenes(device, trained):
    tr = trained[0]
    cold_it, warm_it = 0, 0
    for cfg in synth.cnn_train_configs(count=3, seed0=9000):
        d = synth.make_hsi(cfg)
        v = torch.from_numpy(d["v"]).to(device)
        sv = nt.Solver(*v.shape, 4, 4, device=device)
        ref = sv.solve(v, nt.make_params(max_iter=20000, rel_tol=1e-7, **d["radii"]))[0].clone()
        r = ws.solve_cold_warm(v, d["radii"], tr.params, rel_tol=1e-4, max_iter=5000, solver=sv)
        cold, warm, u0 = r["cold"], r["warm"], r["u0"]
        early = nt.make_params(max_iter=50, **d["radii"])
        dc50 = _dist(sv.solve(v, early)[0], ref)
        dw50 = _dist(sv.solve(v, early, u0=u0)[0], ref)
        print(f"scene {cfg.seed}: estimate {_dist(u0, ref):.2e} vs observation {_dist(v, ref):.2e}; "
              f"after 50 iterations cold {dc50:.2e} warm {dw50:.2e}; to rel-tol 1e-4 cold "
              f"{cold[3]['iters']} warm {warm[3]['iters']} iterations", flush=True)
        assert _dist(u0, ref) <= 0.5 * _dist(v, ref)
        assert dw50 <= dc50 / 3
        assert cold[3]["converged"] and warm[3]["converged"]
        rad = d["radii"]
        assert warm[3]["l1_s"] <= rad["alpha"] * (1 + 1e-5)
        assert warm[3]["l1_t"] <= rad["beta"] * (1 + 1e-5)
        cold_it += cold[3]["iters"]
        warm_it += warm[3]["iters"]
    print(f"total iterations to rel-tol 1e-4: cold {cold_it} warm {warm_it}", flush=True)
    assert warm_it <= 0.85 * cold_it


def test_cold_and_warm_runs_meet(device, trained):
    """Long runs from both starts reach the same point (one solution)."""
    tr = trained[0]
    cfg = synth.HSIConfig(16, 16, 16, endmembers=4, cells=6, sigma=0.05, p_sp=0.05,
                          p_stripe=0.1, seed=9100)
    d = synth.make_hsi(cfg)
    v = torch.from_numpy(d["v"]).to(device)
    sv = nt.Solver(16, 16, 16, 4, 4, device=device)
    prm = nt.make_params(max_iter=30000, **d["radii"])
    uc, sc, tc, _ = sv.solve(v, prm)
    uc, sc, tc = uc.clone(), sc.clone(), tc.clone()
    uw, sw, tw, _ = sv.solve(v, prm, u0=nt.cnn_forward(tr.params, v))
    du, ds, dt = _dist(uw, uc), _dist(sw, sc), _dist(tw, tc)
    print(f"after 30000 iterations: u {du:.2e} s {ds:.2e} t {dt:.2e}", flush=True)
    assert du <= 1e-3 and ds <= 1e-2 and dt <= 1e-2


def test_noise_levels_of_the_large_scene_recorded(device, trained):
    """Held-out 64^3 scenes at the noise levels of the 512 x 512 x 191 warm-start scene
    (Gaussian 0.1, salt-and-pepper 0.1, stripes 0.1): iterations to rel-tol 1e-4 from zero and
    from the estimate are recorded. At these levels the learned start does not reliably need
    fewer iterations (on the large scene it needs more: the stop rule fires at different kinds
    of points for the two starts), so what is asserted is only what holds: the estimate is
    closer to the solution than the observation, both runs converge and stay feasible."""
    tr = trained[0]
    totals = {"cold": 0, "warm": 0}
    for i in range(3):
        cfg = synth.HSIConfig(64, 64, 64, endmembers=8, cells=16, sigma=0.1, p_sp=0.1,
                              p_stripe=0.1, seed=9200 + i)
        d = synth.make_hsi(cfg)
        v = torch.from_numpy(d["v"]).to(device)
        sv = nt.Solver(*v.shape, 4, 4, device=device)
        ref = sv.solve(v, nt.make_params(max_iter=20000, rel_tol=1e-7, **d["radii"]))[0].clone()
        r = ws.solve_cold_warm(v, d["radii"], tr.params, rel_tol=1e-4, max_iter=8000, solver=sv)
        cold, warm, u0 = r["cold"], r["warm"], r["u0"]
        print(f"scene {cfg.seed} (noise 0.1 / 0.1 / 0.1): estimate {_dist(u0, ref):.2e} vs "
              f"observation {_dist(v, ref):.2e}; to rel-tol 1e-4 cold {cold[3]['iters']} "
              f"(distance {_dist(cold[0], ref):.2e}) warm {warm[3]['iters']} "
              f"(distance {_dist(warm[0], ref):.2e}) iterations", flush=True)
        assert _dist(u0, ref) <= 0.5 * _dist(v, ref)
        assert cold[3]["converged"] and warm[3]["converged"]
        rad = d["radii"]
        assert warm[3]["l1_s"] <= rad["alpha"] * (1 + 1e-5)
        assert warm[3]["l1_t"] <= rad["beta"] * (1 + 1e-5)
        totals["cold"] += cold[3]["iters"]
        totals["warm"] += warm[3]["iters"]
    print(f"total iterations to rel-tol 1e-4 at these noise levels: {totals}", flush=True)
