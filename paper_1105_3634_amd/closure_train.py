"""Training of the force-closure network on data from the plain solver.

Snapshots come from the GPU solver itself: seeded initial states of a
binary mixture are advanced with the exact force, and every `sample_every`
steps the state and its exact force are taken as one training pair
(mlb_closure_sample).  The pairs stay in device memory as a pool; training
then runs shuffled epochs over the pool, one Adam step per pair
(mlb_net_train_step), each on the pair's relative squared error (the loss
divided by the target's mean square, the measure the closure's exact-force
checks use).

The scales fix the network's units: n_ref is the mean species density of
the first state, j_ref and f_ref are the RMS momentum density and force
over the pool, so inputs and targets are O(1).  The pool's sums, its
rescaling and the error measure run in the library (mlb_net_pool_stats,
mlb_net_pool_rescale, mlb_net_rel_error); this module only sequences calls
and keeps the pool's device tensors.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Callable, List, Optional, Sequence

import numpy as np

from . import GpuMixture, GpuNet


@dataclasses.dataclass
class TrainReport:
    samples: int
    steps: int
    losses: List[float]
    scales: tuple
    collect_seconds: float
    train_seconds: float


def init_params(seed: int = 0, channels=(14, 32, 32, 32, 6)):
    """Uniform He initialisation (fan-in 27 Ci), zero biases; PCG64-seeded."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for ci, co in zip(channels[:-1], channels[1:]):
        lim = math.sqrt(6.0 / (27 * ci))
        out.append({"W": rng.uniform(-lim, lim, size=(co, ci, 3, 3, 3)), "b": np.zeros(co)})
    return out


def collect(net: GpuNet, states: Sequence[Callable[[], tuple]], per_state: int, sample_every: int,
            n_ref: float, device: str = "cuda:0"):
    """Training pairs with input scales (n_ref, 1) and unit force scale: for
    every initial state, `per_state` snapshots taken every `sample_every`
    steps from step 0 on.  Returns device tensors x [S][14][...], t [S][6][...]."""
    import torch

    net.set_scales(n_ref, 1.0, 1.0)
    xs, ts = [], []
    for make in states:
        mix, n0, u0 = make()
        g = GpuMixture(mix, n0, u0, precision=32, device=device)
        for _ in range(per_state):
            x, t = g.closure_sample(net)
            xs.append(x)
            ts.append(t)
            g.step(sample_every)
        del g
    torch.cuda.synchronize()
    return torch.stack(xs), torch.stack(ts)


def fit(net: GpuNet, x, t, epochs: int, lr: float = 1e-3, lr_final: float = 1e-5, seed: int = 0,
        log_every: int = 0, log: Optional[Callable[[str], None]] = None) -> List[float]:
    """Shuffled epochs over scaled pairs x [S][14][...], t [S][6][...]; the
    learning rate decays geometrically from lr to lr_final over all steps."""
    import torch

    S = x.shape[0]
    total = epochs * S
    decay = (lr_final / lr) ** (1.0 / max(1, total - 1))
    # each pair's loss is divided by its target's mean square (library sums)
    _, target_ms = net.pool_stats(x, t)
    wts = [1.0 / max(v, 1e-300) for v in target_ms]
    rng = np.random.Generator(np.random.PCG64(seed))
    losses = []
    k = 0
    for ep in range(epochs):
        for i in rng.permutation(S):
            want = log is not None and log_every > 0 and (k % log_every == 0 or k == total - 1)
            loss, _ = net.train_step(x[i], t[i], lr=lr * decay ** k, want_loss=want, loss_weight=wts[i])
            if want:
                losses.append(loss)
                log(f"step {k} (epoch {ep}): relative loss {loss:.4e}")
            k += 1
    torch.cuda.synchronize()
    return losses


def prepare_pool(net: GpuNet, states: Sequence[Callable[[], tuple]], per_state: int = 100, sample_every: int = 10,
                 device: str = "cuda:0"):
    """Collect pairs from `states` (callables returning (mixture, n0, u0) on
    the net's grid) and fix the scales from them: returns the rescaled pool
    (x, t), the scales (n_ref, j_ref, f_ref), already set on `net`, and the
    collection time."""
    t0 = time.perf_counter()
    _, n0, _ = states[0]()
    n_ref = float(np.mean(n0))
    x, t = collect(net, states, per_state, sample_every, n_ref, device)
    j_ms, t_ms = net.pool_stats(x, t)
    j_ref = max(math.sqrt(j_ms), 1e-30)
    f_ref = max(math.sqrt(sum(t_ms) / len(t_ms)), 1e-30)
    net.pool_rescale(x, t, j_ref, f_ref)
    scales = (n_ref, j_ref, f_ref)
    net.set_scales(*scales)
    return x, t, scales, time.perf_counter() - t0


def train_closure(net: GpuNet, states: Sequence[Callable[[], tuple]], per_state: int = 100, sample_every: int = 10,
                  epochs: int = 10, lr: float = 1e-3, lr_final: float = 1e-5, seed: int = 0,
                  log_every: int = 0, log: Optional[Callable[[str], None]] = None,
                  device: str = "cuda:0") -> TrainReport:
    """Collect pairs from `states`, fix the scales from them, and fit the network."""
    x, t, scales, collect_s = prepare_pool(net, states, per_state, sample_every, device)
    t1 = time.perf_counter()
    losses = fit(net, x, t, epochs, lr, lr_final, seed, log_every, log)
    return TrainReport(samples=int(x.shape[0]), steps=epochs * int(x.shape[0]), losses=losses, scales=scales,
                       collect_seconds=collect_s, train_seconds=time.perf_counter() - t1)


def closure_error(net: GpuNet, g: GpuMixture) -> float:
    """Relative L2 error of the network's force against the exact force in the
    current state of mixture `g` (same grid as `net`)."""
    x, t = g.closure_sample(net)
    return net.rel_error(net.forward(x), t)
