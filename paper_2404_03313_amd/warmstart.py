"""Learned initial estimate for Alg. 1: training-pair generation with the batched solver,
training of the network through s3ttv_cnn_train_step, and cold-vs-warm solves.

Every numeric step runs in the library (solver, network forward/backward, Adam); this module
only sequences calls, draws seeded mini-batch orders and moves tensors.
"""
from __future__ import annotations

import concurrent.futures as cf
import time
from typing import List, Optional

import numpy as np

from . import native as nt
from . import synth


def _torch():
    import torch
    return torch


def make_pairs(cfgs: List[synth.HSIConfig], k=(4, 4), rel_tol: float = 1e-5,
               max_iter: int = 3000, group: int = 16, device="cuda", log=None):
    """Observations v and P-PDS solutions u* (the training targets) for every config, as two
    (n, n1, n2, n3) float32 device tensors (all configs must share one shape)."""
    torch = _torch()
    n = len(cfgs)
    shape = (cfgs[0].n1, cfgs[0].n2, cfgs[0].n3)
    V = torch.empty((n,) + shape, dtype=torch.float32, device=device)
    U = torch.empty_like(V)
    ws = None
    iters = []
    t0 = time.time()
    starts = list(range(0, n, group))
    # the host builds the next group's scenes while the device solves the current one
    ex = cf.ThreadPoolExecutor(max_workers=4)
    pending = [ex.submit(synth.make_hsi, c) for c in cfgs[:group]]
    for gi, g0 in enumerate(starts):
        data = [f.result() for f in pending]
        nxt = cfgs[g0 + group:g0 + 2 * group]
        pending = [ex.submit(synth.make_hsi, c) for c in nxt]
        probs = []
        for i, d in enumerate(data, start=g0):
            V[i].copy_(torch.from_numpy(d["v"]))
            prm = nt.make_params(max_iter=max_iter, rel_tol=rel_tol, **d["radii"])
            probs.append(dict(v=V[i], k1=k[0], k2=k[1], params=prm))
        res, _ = nt.solve_batched(probs, workspace=ws)
        if ws is None:
            ws = nt._workspace(nt.batch_workspace_bytes([(*shape, k[0], k[1])] * len(probs)),
                               V.device)
        for i, (u, _, _, st) in enumerate(res):
            U[g0 + i].copy_(u)
            iters.append(st["iters"])
        if log:
            log(f"pairs {min(n, g0 + group)}/{n}: {time.time() - t0:.1f} s, "
                f"mean iterations {np.mean(iters):.0f}")
    ex.shutdown()
    return V, U, iters


class Trainer:
    """Adam training of the network on (v, u*) pairs held on the device."""

    def __init__(self, params: np.ndarray, device="cuda"):
        torch = _torch()
        self.params = torch.from_numpy(np.asarray(params, dtype=np.float32)).to(device)
        self.m = torch.zeros_like(self.params)
        self.v2 = torch.zeros_like(self.params)
        self.step = 0
        self.ws = None

    def train(self, V, U, steps: int, batch: int = 8, lr: float = 1e-3, seed: int = 0,
              lr_final: Optional[float] = None, log=None, log_every: int = 50):
        """`steps` Adam steps on seeded mini-batches (each epoch a fresh permutation); the
        learning rate decays by cosine to lr_final (default lr / 10). Returns the losses."""
        torch = _torch()
        rng = np.random.Generator(np.random.PCG64(seed))
        n = V.shape[0]
        lr_final = lr / 10 if lr_final is None else lr_final
        order = rng.permutation(n)
        pos = 0
        losses = []
        t0 = time.time()
        for k in range(steps):
            if pos + batch > n:
                order, pos = rng.permutation(n), 0
            idx = torch.from_numpy(order[pos:pos + batch].astype(np.int64)).to(V.device)
            pos += batch
            vb = V.index_select(0, idx).contiguous()
            ub = U.index_select(0, idx).contiguous()
            if self.ws is None:
                self.ws = nt._workspace(nt.cnn_workspace_bytes(vb.shape, True), V.device)
            rate = lr_final + 0.5 * (lr - lr_final) * (1 + np.cos(np.pi * k / max(steps, 1)))
            self.step += 1
            losses.append(nt.cnn_train_step(self.params, self.m, self.v2, self.step, rate, vb,
                                            ub, workspace=self.ws))
            if log and (k + 1) % log_every == 0:
                log(f"step {k + 1}/{steps}: loss {np.mean(losses[-log_every:]):.3e} "
                    f"({time.time() - t0:.1f} s)")
        return losses

    def loss(self, V, U, batch: int = 8):
        """Mean loss over all pairs (forward and backward, no update)."""
        tot = 0.0
        for a in range(0, V.shape[0], batch):
            vb, ub = V[a:a + batch].contiguous(), U[a:a + batch].contiguous()
            tot += nt.cnn_grad(self.params, vb, ub)[0] * vb.shape[0]
        return tot / V.shape[0]


def solve_cold_warm(v, radii: dict, params, k=(4, 4), rel_tol: float = 1e-4,
                    max_iter: int = 5000, solver: Optional[nt.Solver] = None):
    """Solve one scene from u0 = 0 and from u0 = v + f(v); returns a dict with both results,
    their statistics and the network's own time (the warm time includes it)."""
    torch = _torch()
    n1, n2, n3 = v.shape
    sv = solver or nt.Solver(n1, n2, n3, k[0], k[1], device=v.device)
    prm = nt.make_params(max_iter=max_iter, rel_tol=rel_tol, **radii)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cold = sv.solve(v, prm)
    torch.cuda.synchronize()
    t_cold = time.perf_counter() - t0
    ws = nt._workspace(nt.cnn_workspace_bytes(v.shape, False), v.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u0 = nt.cnn_forward(params, v, workspace=ws)
    torch.cuda.synchronize()
    t_net = time.perf_counter() - t0
    warm = sv.solve(v, prm, u0=u0)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    return dict(cold=cold, warm=warm, u0=u0, t_cold=t_cold, t_warm=t_warm, t_net=t_net)
