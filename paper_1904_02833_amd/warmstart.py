"""Learned warm start: record the solver's own multipliers, train the network
on the GPU with the library's BF16-MFMA kernels, and load it into a solver.

Recording runs a "teacher" copy of a batch with a tight tolerance, so the
targets are the multipliers the plain method converges to from each
substep's predicted state.  Training is mean-squared error with Adam on
mini-batches.  Torch only holds the buffers; every arithmetic step (inputs,
solves, forward, backward, optimiser, statistics) runs in the library.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import Net, Sim, WARM_MLP


@dataclasses.dataclass
class Dataset:
    features: object  # torch [rows, 32], device
    targets: object   # torch [rows, 3], device


def record(wl, n_steps, warmup_steps=0, tol=1e-6, iters=2000, device="cuda", **over) -> Dataset:
    """Run the batch `wl` for warmup_steps with its own settings, then record
    n_steps steps solved to `tol` (at most `iters` iterations per substep)."""
    import torch

    if warmup_steps:
        lead = Sim(wl, device=device, **over)
        lead.step(warmup_steps)
        state = lead.read()
        lead.close()
    teacher = Sim(wl, device=device, tol=tol, iters=iters, **over)
    if warmup_steps:
        teacher.write(**state)
    rows = teacher.record_rows(n_steps)
    feats = torch.empty((rows, 32), dtype=torch.float32, device=device)
    tgts = torch.empty((rows, 3), dtype=torch.float32, device=device)
    written = teacher.step_record(n_steps, feats, tgts)
    assert written == rows
    teacher.close()
    return Dataset(feats, tgts)


def record_on_policy(wl, n_records, stride=1, warmup_steps=0, tol=1e-6, iters=2000, device="cuda",
                     **over) -> Dataset:
    """Targets at the states the deployed (plain) solver visits: the batch
    advances with its own settings; every `stride` steps a teacher copy
    solves the next step's first substep from that state to `tol`, and only
    that substep's rows are kept."""
    import torch

    lead = Sim(wl, device=device, **over)
    teacher = Sim(wl, device=device, tol=tol, iters=iters, **over)
    per_sub = 2 * teacher.J
    rows = teacher.record_rows(1)
    f = torch.empty((rows, 32), dtype=torch.float32, device=device)
    t = torch.empty((rows, 3), dtype=torch.float32, device=device)
    feats, tgts = [], []
    if warmup_steps:
        lead.step(warmup_steps)
    for _ in range(n_records):
        teacher.write(**lead.read())
        teacher.step_record(1, f, t)
        feats.append(f[:per_sub].clone())
        tgts.append(t[:per_sub].clone())
        lead.step(stride)
    lead.close()
    teacher.close()
    return Dataset(torch.cat(feats), torch.cat(tgts))


def concat(parts) -> Dataset:
    import torch
    return Dataset(torch.cat([p.features for p in parts]), torch.cat([p.targets for p in parts]))


def shuffled(ds: Dataset, seed: int) -> Dataset:
    """One host-side permutation of the rows (a data-loading step), uploaded
    back so training can take contiguous mini-batches."""
    import torch
    rng = np.random.default_rng(seed)
    perm = rng.permutation(ds.features.shape[0])
    f = torch.as_tensor(ds.features.cpu().numpy()[perm]).to(ds.features.device)
    t = torch.as_tensor(ds.targets.cpu().numpy()[perm]).to(ds.targets.device)
    return Dataset(f.contiguous(), t.contiguous())


def train(ds: Dataset, epochs=3, batch=4096, lr=1e-3, seed=0, init_scale=0.1, log=None) -> Net:
    """Adam on mean-squared error over contiguous mini-batches of a shuffled
    copy of the dataset.  Returns the trained network."""
    import torch

    data = shuffled(ds, seed)
    rng = np.random.default_rng(seed + 1)
    P = 6467
    # fan-in scaled initial weights, zero biases
    p = np.zeros(P, np.float32)
    p[0:2048] = rng.normal(scale=init_scale * np.sqrt(2.0 / 32), size=2048)
    p[2112:6208] = rng.normal(scale=init_scale * np.sqrt(2.0 / 64), size=4096)
    p[6272:6464] = rng.normal(scale=init_scale * np.sqrt(1.0 / 64), size=192)
    ms = Net.norm_stats(data.features)
    net = Net(p, ms, device=data.features.device)
    n = data.features.shape[0]
    nb = max(1, n // batch)
    order = np.arange(nb)
    for ep in range(epochs):
        rng.shuffle(order)
        for k in order:
            a, b = int(k) * batch, min(n, int(k + 1) * batch)
            g, loss = net.grad(data.features[a:b], data.targets[a:b])
            net.adam(g, lr=lr)
        if log is not None:
            _, l_all = net.grad(data.features[: min(n, 1 << 18)], data.targets[: min(n, 1 << 18)])
            log(ep, float(l_all.cpu()))
    torch.cuda.synchronize()
    return net


def evaluate_loss(net: Net, ds: Dataset) -> float:
    _, l = net.grad(ds.features, ds.targets)
    return float(l.cpu())


def learned_sim(wl, net: Net, device="cuda", fallback=1, **over) -> Sim:
    sim = Sim(wl, device=device, warm_start=WARM_MLP, mlp_fallback=fallback, **over)
    sim.set_mlp(net.params, net.mean_std)
    return sim
