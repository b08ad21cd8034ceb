"""FP64 CPU oracle of the convolutional initial-estimate network — TEST INFRASTRUCTURE.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this module. It shares no code with the GPU library.

The network computes a start for Alg. 1 (whose initial values are free; Prob. (18) is
convex, so the start only changes the iteration count): u0 = v + f(v) with
f = C4 o R o C3 o R o C2 o R o C1 o R o C0, each C a 3x3x3 convolution with bias over
(i, j, b) with zero padding, channels 1 -> 32 -> 32 -> 32 -> 32 -> 1, R = ReLU.
The training loss is the mean of (u0 - target)^2 over all voxels; the optimizer is Adam.

Data: volumes are float64 arrays of shape (nb, n1, n2, n3); hidden activations are
(nb, n1, n2, n3, channels). Parameters are one flat vector: per layer the weights
[27][cout][cin] (tap t = (di+1)*9 + (dj+1)*3 + (db+1) reads the input at (i+di, j+dj, b+db))
followed by the cout biases.

Two arithmetic modes:
  * ``exact``: every value in float64.
  * ``bf16``: float64 sums, but with the values rounded to bfloat16 (round to nearest even)
    where the GPU path stores them in that format: the weights of all layers (biases are kept),
    the four hidden activations, and the four hidden-layer gradients. The remaining
    difference to the GPU path is the FP32 summation order.
A callable may be given instead of a mode name: it is applied at the same storage points in
place of the bfloat16 rounding (the tests pass random relative perturbations of the size of a
bfloat16 rounding error, to measure how such errors propagate to the outputs).
"""
from __future__ import annotations

import numpy as np

CHANNELS = (1, 32, 32, 32, 32, 1)
TAPS = [(di, dj, db) for di in (-1, 0, 1) for dj in (-1, 0, 1) for db in (-1, 0, 1)]


def layer_sizes():
    """(cin, cout) of the five layers."""
    return [(CHANNELS[l], CHANNELS[l + 1]) for l in range(5)]


def param_count() -> int:
    return sum(27 * ci * co + co for ci, co in layer_sizes())


def unpack(params):
    """Flat parameter vector -> [(W (27, cout, cin), b (cout,))] per layer."""
    params = np.asarray(params, dtype=np.float64)
    assert params.shape == (param_count(),)
    out, off = [], 0
    for ci, co in layer_sizes():
        W = params[off:off + 27 * co * ci].reshape(27, co, ci)
        off += 27 * co * ci
        b = params[off:off + co]
        off += co
        out.append((W, b))
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def bf16_round(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even) via the float32 bit pattern; float64 out."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _shift(xp, di, dj, db, n1, n2, n3):
    """From a volume zero-padded by one on axes 1..3, the view x[i+di, j+dj, b+db]."""
    return xp[:, 1 + di:1 + di + n1, 1 + dj:1 + dj + n2, 1 + db:1 + db + n3]


def _pad(x):
    return np.pad(x, [(0, 0), (1, 1), (1, 1), (1, 1)] + [(0, 0)] * (x.ndim - 4))


def conv(x, W, b):
    """y[p][co] = b[co] + sum_t sum_ci W[t][co][ci] x[p + off_t][ci], zero outside a volume.
    x: (nb, n1, n2, n3, cin); returns (nb, n1, n2, n3, cout)."""
    nb, n1, n2, n3, _ = x.shape
    xp = _pad(x)
    y = np.broadcast_to(b, (nb, n1, n2, n3, W.shape[1])).copy()
    for t, (di, dj, db) in enumerate(TAPS):
        y += _shift(xp, di, dj, db, n1, n2, n3) @ W[t].T
    return y


def conv_adj(g, W):
    """Adjoint of x -> conv(x, W, 0): dx[p][ci] = sum_t sum_co W[t][co][ci] g[p - off_t][co]."""
    nb, n1, n2, n3, _ = g.shape
    gp = _pad(g)
    dx = np.zeros((nb, n1, n2, n3, W.shape[2]))
    for t, (di, dj, db) in enumerate(TAPS):
        dx += _shift(gp, -di, -dj, -db, n1, n2, n3) @ W[t]
    return dx


def conv_wgrad(x, g):
    """Derivative of <g, conv(x, W, b)> in W and b:
    dW[t][co][ci] = sum_p g[p][co] x[p + off_t][ci], db[co] = sum_p g[p][co]."""
    nb, n1, n2, n3, ci = x.shape
    co = g.shape[-1]
    xp = _pad(x)
    G = g.reshape(-1, co)
    dW = np.empty((27, co, ci))
    for t, (di, dj, db) in enumerate(TAPS):
        dW[t] = G.T @ _shift(xp, di, dj, db, n1, n2, n3).reshape(-1, ci)
    return dW, G.sum(axis=0)


def forward(params, v, mode: str = "exact"):
    """u0 = v + f(v). v: (nb, n1, n2, n3) (or one (n1, n2, n3) volume). Returns (u0, cache)."""
    assert callable(mode) or mode in ("exact", "bf16")
    v = np.asarray(v, dtype=np.float64)
    single = v.ndim == 3
    if single:
        v = v[None]
    rnd = mode if callable(mode) else (bf16_round if mode == "bf16" else (lambda a: a))
    layers = [(rnd(W), b) for W, b in unpack(params)]
    acts = []
    x = v[..., None]
    for l in range(4):
        x = rnd(np.maximum(conv(x, *layers[l]), 0.0))
        acts.append(x)
    u = v + conv(x, *layers[4])[..., 0]
    cache = {"v": v, "acts": acts, "layers": layers, "rnd": rnd}
    return (u[0] if single else u), cache


def loss_grad(params, v, target, mode: str = "exact"):
    """Loss mean((u0 - target)^2) and its gradient in the parameters (at the weights the mode
    uses). Returns (loss, grad vector)."""
    u, c = forward(params, v, mode)
    target = np.asarray(target, dtype=np.float64)
    if target.ndim == 3:
        target, u = target[None], u[None]
    d = u - target
    n = d.size
    loss = float(np.sum(d * d) / n)
    du = (2.0 / n) * d[..., None]
    acts, layers, rnd = c["acts"], c["layers"], c["rnd"]
    grads = [None] * 5
    grads[4] = conv_wgrad(acts[3], du)
    g = rnd(conv_adj(du, layers[4][0]) * (acts[3] > 0))
    for l in (3, 2, 1):
        grads[l] = conv_wgrad(acts[l - 1], g)
        g = rnd(conv_adj(g, layers[l][0]) * (acts[l - 1] > 0))
    grads[0] = conv_wgrad(c["v"][..., None], g)
    return loss, pack(grads)


def adam(params, m, v2, g, step: int, lr: float, b1: float = 0.9, b2: float = 0.999,
         eps: float = 1e-8):
    """One bias-corrected Adam step; returns (params, m, v2)."""
    m = b1 * m + (1 - b1) * g
    v2 = b2 * v2 + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v2 / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v2
