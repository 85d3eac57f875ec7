"""Training data and training loop of the learned correction network.

Pairs come from the plain solver: restarted A_0-preconditioned GMRES(m) is run one cycle
at a time from x = 0; after every cycle the iterate x_k gives the pair
(r_k, e_k) = (b - A x_k, x* - x_k), with A e_k = r_k, where x* is the converged FP64
solution.  The network is trained to map r_k to e_k - A_0^{-1} r_k (sg_net_train_pairs).
Everything runs on the GPU through the native library.
"""
from __future__ import annotations

import numpy as np

from . import sg


def solver_pairs(op, b, cycle=3, max_pairs=16, tol=1e-11):
    """(r_k, e_k) pairs from the cycles of plain GMRES(cycle) on A x = b (device tensors)."""
    xs, info = op.gmres(b, restart=50, maxit=2000, pc="mean", precision="f64", tol=tol)
    if not info["converged"]:
        raise sg.SGError("reference solve did not converge")
    x = op.empty()
    x.zero_()
    pairs = []
    for _ in range(max_pairs):
        op.gmres(b, x, restart=cycle, maxit=cycle, pc="mean", precision="f64", tol=1e-300, x0_zero=False)
        r = sg.axpby(1.0, b, -1.0, op.apply(x))
        e = sg.axpby(1.0, xs, -1.0, x)
        if sg.norm(r) <= 1e-9 * sg.norm(b):
            break
        pairs.append((r, e))
    return pairs


def train(net, samples, steps, batch=8, lr=1e-3, precision="f64", seed=0, log=None):
    """Adam on random mini-batches of `samples` = [(op, r, e)] (all ops on one grid size);
    returns the list of mini-batch losses."""
    rng = np.random.default_rng(seed)
    losses = []
    for it in range(steps):
        idx = rng.choice(len(samples), size=min(batch, len(samples)), replace=False)
        ops = [samples[i][0] for i in idx]
        losses.append(net.train_pairs(ops, [samples[i][1] for i in idx], [samples[i][2] for i in idx], lr,
                                      precision))
        if log and (it % 50 == 0 or it == steps - 1):
            log("train step %d: loss %.4e" % (it, losses[-1]))
    return losses
