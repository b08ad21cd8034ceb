"""What the learned initial estimate gains (GPU). The network is trained by the library's
own kernels on solver-generated pairs; held-out scenes are then solved to rel-tol 1e-4 from
u0 = 0 and from u0 = v + f(v). Prob. (18) is convex, so both runs approach one solution: the
zero-start run is the judge of the warm-started one."""
import numpy as np
import pytest
import torch

from paper_2404_03313_amd import native as nt
from paper_2404_03313_amd import synth
from paper_2404_03313_amd import warmstart as ws

pytestmark = pytest.mark.gpu


def test_trained_network_reduces_iterations_to_tolerance(device):
    print("pairs: 64 scenes 64^3", flush=True)
    V, U, _ = ws.make_pairs(synth.cnn_train_configs(count=64), rel_tol=1e-5, max_iter=3000,
                            device=device)
    tr = ws.Trainer(synth.cnn_init(0), device=device)
    before = tr.loss(V, U)
    losses = tr.train(V, U, steps=300, batch=8, lr=1e-3)
    after = tr.loss(V, U)
    print(f"training loss {before:.3e} -> {after:.3e}", flush=True)
    assert after < 0.2 * before
    assert np.isfinite(losses).all()
    del V, U
    cold_it, warm_it = 0, 0
    for cfg in synth.cnn_train_configs(count=3, seed0=9000):
        d = synth.make_hsi(cfg)
        v = torch.from_numpy(d["v"]).to(device)
        r = ws.solve_cold_warm(v, d["radii"], tr.params, rel_tol=1e-4, max_iter=5000)
        ref = nt.solve(v, 4, 4, max_iter=20000, rel_tol=1e-7, **d["radii"])[0]
        cold, warm = r["cold"], r["warm"]
        dc = float((cold[0] - ref).norm() / ref.norm())
        dw = float((warm[0] - ref).norm() / ref.norm())
        print(f"scene {cfg.seed}: iterations cold {cold[3]['iters']} warm {warm[3]['iters']}, "
              f"distance to the rel-tol 1e-7 solution cold {dc:.2e} warm {dw:.2e}", flush=True)
        assert cold[3]["converged"] and warm[3]["converged"]
        # the warm-started result is at least as good a solution as the zero-start one
        assert dw <= 1.5 * dc + 1e-3
        # constraints of Prob. (18): the l1 balls hold exactly (s and t are projections), the
        # fidelity ball as closely as for the zero-start result
        rad = d["radii"]
        assert warm[3]["l1_s"] <= rad["alpha"] * (1 + 1e-5)
        assert warm[3]["l1_t"] <= rad["beta"] * (1 + 1e-5)
        assert warm[3]["fid"] <= max(cold[3]["fid"], rad["eps"]) * 1.02
        cold_it += cold[3]["iters"]
        warm_it += warm[3]["iters"]
    print(f"total iterations cold {cold_it} warm {warm_it}", flush=True)
    assert warm_it <= 0.85 * cold_it
