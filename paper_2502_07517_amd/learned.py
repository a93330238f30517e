"""Training workflow of the learned troubled-cell indicator over the C ABI.

The pairs come from the method itself: before each step of a run that uses
the smoothness indicator, ``Solver.features`` returns every element's
modal-energy features and the indicator's blending coefficient for the state
that step will limit.  ``train_indicator`` fits a network to those pairs with
the library's GPU training kernels (``crkfr_mlp_train``).  This module only
orders calls and moves rows between device buffers; the features, the
network and its training run in the HIP library.
"""
import numpy as np

from . import crkfr as C


def collect_pairs(solvers, steps, every=1):
    """Step each solver (already holding a state and the smoothness indicator)
    `steps` times, keeping the (features, alpha) pairs of every `every`-th
    step.  Returns float32 CUDA tensors X [rows, N] and y [rows]."""
    import torch
    xs, ys = [], []
    for s in solvers:
        for k in range(steps):
            if k % every == 0:
                f, a = s.features(device=True)
                xs.append(f)
                ys.append(a.to(torch.float32))
            s.step(0.0)
    return torch.cat(xs), torch.cat(ys)


def pairs_of_states(solver, states):
    """(features, alpha) of each given state (set on `solver`, whose
    configuration fixes the equation and degree), concatenated."""
    import torch
    xs, ys = [], []
    for u in states:
        solver.set_state(u)
        f, a = solver.features(device=True)
        xs.append(f)
        ys.append(a.to(torch.float32))
    return torch.cat(xs), torch.cat(ys)


def train_indicator(X, y, *, hidden=16, epochs=30, batch=4096, lr=3e-3, seed=0, margin=0.02):
    """Fit a network to the pairs (rows shuffled once with a seeded
    permutation); the feature box is the data's range widened by `margin`.
    Returns (Mlp, per-epoch mean loss)."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(int(seed))
    perm = torch.randperm(X.shape[0], generator=g).to(X.device)
    Xs, ys = X[perm].contiguous(), y[perm].contiguous()
    net = C.Mlp(X.shape[1], hidden, seed=seed)
    net.fit_box(Xs, margin)
    hist = net.train(Xs, ys, epochs=epochs, batch=batch, lr=lr)
    return net, hist


def agreement(net, X, y, alpha_min=1e-3, alpha_max=1.0, within=None):
    """Share of rows on which the network and the labels agree about
    'troubled' (alpha > 0 after the indicator's clipping), and the mean
    absolute difference of the clipped coefficients; with `within`, also the
    share of rows whose coefficients differ by at most that much."""
    out = net.forward(X).double().cpu().numpy()
    a = np.where(out < alpha_min, 0.0, np.minimum(out, alpha_max))
    t = y.double().cpu().numpy()
    res = (float(np.mean((a > 0) == (t > 0))), float(np.mean(np.abs(a - t))))
    if within is not None:
        res += (float(np.mean(np.abs(a - t) <= within)),)
    return res
