"""Training data and training loop of the learned screen.

Orchestration only: the labels come from the library's own transient runs
(trees-only batches with the currents of an IR solve held fixed, stepped past
the horizon of interest), the features from its feature kernel, and every
forward, backward and Adam step from its MLP kernels.  Minibatches are
assembled by slicing device tensors.
"""
from __future__ import annotations

import time

import numpy as np

from . import synth
from ._binding import MLP, Batch

T_REF = 1e8   # s; the model predicts log10(t_nuc / T_REF)


def fixed_j_grid(grid, mat, run, factor: float = 1.0):
    """The trees-only copy of ``grid`` with the currents of its t = 0 IR
    solve (times ``factor``)."""
    B = Batch(grid, mat, dict(run, screen=0))
    try:
        B.ir_solve()
        j = B.seg_j(0)
    finally:
        B.close()
    return synth.with_prescribed_j(grid, j * factor)


def label_cap(run, horizon_steps: int) -> float:
    """The label of a tree that had not nucleated within the label horizon."""
    return float(np.log10(horizon_steps * float(run["dt"]) / T_REF))


def label_batch(grid_fixed_j, mat, run, mc, horizon_steps: int, chunk: int = 1000):
    """Features and labels of every steady-state-mortal (tree, sample) of a
    trees-only grid: label = log10(min(t_nuc, horizon) / T_REF) with
    t_nuc = (first nucleation step + 1) dt.  Returns (X device [m][12],
    y device [m], info dict)."""
    import torch
    t0 = time.perf_counter()
    B = Batch(grid_fixed_j, mat, run, mc)
    try:
        mortal = B.screen()                       # [S][n_trees]; only mortal trees are stepped
        X = B.features()                          # rows tree * S + sample
        done = 0
        while done < horizon_steps:
            n = min(chunk, horizon_steps - done)
            B.stress_step(n)
            done += n
        first = B.first_nucleation()              # [S][n_trees]
        info = B.info()
    finally:
        B.close()
    S, nt = mortal.shape
    dt = float(run["dt"])
    t_nuc = np.where(first >= 0, (first + 1.0) * dt, horizon_steps * dt)
    t_nuc = np.minimum(t_nuc, horizon_steps * dt)
    rows = (np.arange(nt)[None, :] * S + np.arange(S)[:, None])       # [S][nt]
    sel = mortal.astype(bool)
    idx = torch.as_tensor(rows[sel].astype(np.int64), device="cuda")
    y = torch.as_tensor(np.log10(t_nuc[sel] / T_REF), dtype=torch.float32, device="cuda")
    info = dict(n_pairs=int(sel.sum()), n_censored=int(((first < 0) & sel).sum()),
                node_steps=info["node_steps"], wall_s=time.perf_counter() - t0)
    return X[idx].contiguous(), y, info


def training_set(seed: int, n_grids: int, mat, run, n_samples: int, horizon_steps: int,
                 cov=(0.2, 0.2), n: int = 200, log=None, family: str = "sparse_via"):
    """Concatenated (X, y) over ``n_grids`` random grids of a family (the
    200x200 sparse-via grids, the long-line grids with ``family="lines"``, or
    the cold long-line grids with ``family="cold_lines"``),
    each with ``n_samples`` Monte Carlo samples of the diffusivity and
    critical stress."""
    import torch
    Xs, ys, infos = [], [], []
    if family == "lines":
        grids = synth.line_training_grids(seed, n_grids)
    elif family == "cold_lines":
        grids = synth.line_training_grids(seed, n_grids, cold=True)
    else:
        grids = synth.screen_training_grids(seed, n_grids, n=n)
    for k, (g, factor) in enumerate(grids):
        gj = fixed_j_grid(g, mat, run, factor)
        mc = dict(n_samples=n_samples, seed=seed * 1000 + k, cov_kappa=cov[0], cov_scrit=cov[1])
        X, y, info = label_batch(gj, mat, dict(run, screen=1), mc, horizon_steps)
        Xs.append(X)
        ys.append(y)
        infos.append(info)
        if log:
            log(f"labels: grid {k + 1}/{n_grids}: {info['n_pairs']} pairs, {info['wall_s']:.2f} s")
    return torch.cat(Xs), torch.cat(ys), infos


def train(mlp: MLP, X, y, steps: int, batch: int = 4096, lr: float = 1e-3, seed: int = 0,
          lr_final: float | None = None):
    """``steps`` Adam steps on minibatches drawn from shuffled passes over
    (X, y) (the ragged tail of each pass is dropped); the learning rate
    decays geometrically from ``lr`` to ``lr_final``.  Returns the loss of
    the last minibatch."""
    import torch
    n = int(X.shape[0])
    batch = min(batch, n)
    per_pass = max(1, n // batch)
    decay = (lr_final / lr) ** (1.0 / max(steps - 1, 1)) if lr_final else 1.0
    gen = torch.Generator().manual_seed(seed)
    loss = None
    k = 0
    while k < steps:
        perm = torch.randperm(n, generator=gen).to(X.device)
        for b in range(per_pass):
            if k >= steps:
                break
            idx = perm[b * batch:(b + 1) * batch]
            loss = mlp.train_step(X[idx].contiguous(), y[idx].contiguous(), lr * decay ** k,
                                  want_loss=(k == steps - 1))
            k += 1
    return loss


def calibrate(mlp: MLP, Xv, yv, quantile: float = 0.995, y_cap: float | None = None) -> float:
    """Shift the output bias so that the predicted nucleation time is at most
    the label on a ``quantile`` fraction of held-out pairs: the screen then
    errs towards activating trees early.  With ``y_cap`` (the label of the
    label runs' horizon) the pairs whose tree had not nucleated by then are
    left out: their label is a lower bound, and a later prediction is no
    error.  Returns the shift (decades)."""
    pred = mlp.forward(Xv).cpu().numpy().astype(np.float64)
    lab = yv.cpu().numpy().astype(np.float64)
    keep = lab < y_cap - 1e-6 if y_cap is not None else np.ones(lab.size, bool)
    err = pred[keep] - lab[keep]
    shift = float(np.quantile(err, quantile))
    p = mlp.params()
    p[-1] -= shift
    mlp.set_params(p)
    return shift
