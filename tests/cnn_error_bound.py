"""Error bound of the network kernels against the exact FP64 network, derived from the
storage formats of the kernels.

The kernels store the weights, the four hidden activations and the four hidden-layer
gradients in bfloat16 (round to nearest even: every stored value x^ satisfies
|x^ - x| <= u_b |x| with u_b = 2^-8) and sum in FP32 (unit roundoff 2^-24, a factor 2^16
smaller, neglected here). A worst-case elementwise bound that adds these errors with
absolute values grows by the absolute row sum of each layer's weights (about 30 for 864
He-initialised inputs) per layer and is useless after five layers. The rounding errors of
distinct stored values are, however, uncorrelated and of both signs, which is the model of
probabilistic rounding-error analysis (Higham and Mary, SIAM J. Sci. Comput. 2019): each
stored value carries an independent relative error distributed in [-u_b, u_b] (uniformly,
which over-states the variance of round-to-nearest). Under that model the output error of the
network is a sum of many independent terms; its typical size `spread` is measured here by
running the exact FP64 network with such random perturbations at exactly the storage points
(the same points where the oracle's bf16 mode rounds) and taking the root mean square of the
output deviation over the draws. The bound used by the tests is LAMBDA x spread per output
block (u0; each layer's weights; each layer's biases).

Test infrastructure: only tests import this module.
"""
from __future__ import annotations

import numpy as np

from oracle import cnn

U_B = 2.0 ** -8
LAMBDA = 3.0
SAMPLES = 12


def perturbation(rng, u=U_B):
    """Relative errors uniform in [-u, u], drawn independently for every stored value."""
    def rnd(a):
        a = np.asarray(a, dtype=np.float64)
        return a * (1.0 + rng.uniform(-u, u, size=a.shape))
    return rnd


def blocks():
    """(name, start, end) of each layer's weight and bias block in the parameter vector."""
    off = 0
    for ci, co in cnn.layer_sizes():
        yield f"W{ci}->{co}", off, off + 27 * ci * co
        off += 27 * ci * co
        yield f"b{ci}->{co}", off, off + co
        off += co


def forward_spread(params, v, samples=SAMPLES, seed=0):
    """Exact u0 and the RMS over random storage perturbations of ||u0_perturbed - u0||."""
    params = np.asarray(params, dtype=np.float64)
    u0, _ = cnn.forward(params, v, "exact")
    rng = np.random.Generator(np.random.PCG64(seed))
    acc = 0.0
    for _ in range(samples):
        up, _ = cnn.forward(params, v, perturbation(rng))
        acc += float(np.sum((up - u0) ** 2))
    return u0, np.sqrt(acc / samples)


def grad_spread(params, v, target, samples=SAMPLES, seed=0):
    """Exact loss and gradient, and per parameter block the RMS over random storage
    perturbations of the gradient deviation (dict name -> spread), plus that of the loss."""
    params = np.asarray(params, dtype=np.float64)
    loss, g = cnn.loss_grad(params, v, target, "exact")
    rng = np.random.Generator(np.random.PCG64(seed))
    acc = {name: 0.0 for name, _, _ in blocks()}
    acc_loss = 0.0
    for _ in range(samples):
        lp, gp = cnn.loss_grad(params, v, target, perturbation(rng))
        acc_loss += (lp - loss) ** 2
        for name, a, b in blocks():
            acc[name] += float(np.sum((gp[a:b] - g[a:b]) ** 2))
    return loss, g, {k: np.sqrt(x / samples) for k, x in acc.items()}, np.sqrt(acc_loss / samples)
