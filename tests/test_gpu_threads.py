"""Solves from several host threads at once: each thread gets its own streams and timing
events, so concurrent calls on distinct workspaces give bitwise the results of the same
calls made one after another."""
import threading

import numpy as np
import pytest

from paper_2404_03313_amd import native as nt
from paper_2404_03313_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _np(x):
    return x.detach().cpu().numpy()


def _data(device, shape, seed):
    import torch
    cfg = synth.HSIConfig(*shape, endmembers=3, cells=5, sigma=0.08, p_sp=0.05, p_stripe=0.2,
                          seed=seed)
    d = synth.make_hsi(cfg)
    return torch.from_numpy(np.ascontiguousarray(d["v"], dtype=np.float32)).to(device), d["radii"]


def test_concurrent_solves_match_sequential(device):
    _say("concurrent solves from three threads: single (timed), single, batched")
    jobs = []
    # a fused-pass shape with kernel timing on, a ragged shape, and a batched pair
    v0, r0 = _data(device, (24, 20, 16), 21)
    v1, r1 = _data(device, (13, 11, 7), 22)
    v2, r2 = _data(device, (16, 12, 12), 23)

    def single(v, radii, k, timing):
        n1, n2, n3 = v.shape
        sv = nt.Solver(n1, n2, n3, *k, device=v.device)
        prm = nt.make_params(max_iter=60, rel_tol=1e-9, check_every=8,
                             timing_mask=(1 << nt.N_KERNEL_CLASSES) - 1 if timing else 0, **radii)
        return [sv.solve(v, prm)]

    def batched():
        probs = [dict(v=v2, k1=2, k2=2, params=nt.make_params(max_iter=50, **r2)),
                 dict(v=v1, k1=2, k2=3, params=nt.make_params(max_iter=40, **r1))]
        res, _ = nt.solve_batched(probs)
        return res

    jobs = [lambda: single(v0, r0, (3, 3), True), lambda: single(v1, r1, (2, 3), False), batched]
    import torch
    torch.cuda.synchronize()
    seq = [job() for job in jobs]
    torch.cuda.synchronize()

    out = [None] * len(jobs)
    errs = []

    def run(i):
        try:
            for _ in range(2):
                out[i] = jobs[i]()
        except Exception as e:  # reported below
            errs.append(repr(e))

    threads = [threading.Thread(target=run, args=(i,)) for i in range(len(jobs))]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=240)
    assert not any(th.is_alive() for th in threads), "a solve thread did not finish"
    assert not errs, errs
    torch.cuda.synchronize()
    for i, (a_list, b_list) in enumerate(zip(out, seq)):
        assert len(a_list) == len(b_list)
        for a, b in zip(a_list, b_list):
            for name, x, y in zip("ust", a[:3], b[:3]):
                assert np.array_equal(_np(x), _np(y)), (i, name)
            assert a[3]["iters"] == b[3]["iters"], i
    # the timed solve recorded its kernels
    assert sum(out[0][0][3]["kernel_calls"].values()) > 0
