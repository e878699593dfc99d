"""Training the delayed-acceptance surrogate on pairs the chains generate.

1. Plain pCN chains run a burn-in, then record (proposal y', log L(y')) every
   `pair_every` steps (the kernel's pair recorder, BF16 rows, slot-major).
2. The targets are standardised on the device (qst_mlp_targets) and the MLP
   (2D^2+D padded to a multiple of 32 -> 512 -> 512 -> 1, GELU) is trained by
   the library's own forward/backward/Adam kernels on consecutive minibatches
   of rows (each minibatch spans different chains at one recording slot).
3. The network's output is rescaled to log-likelihood units (out_scale = sd,
   out_shift = mean) and frozen: it is the stage-1 surrogate of a delayed-
   acceptance run (qst_run_desc.surrogate).

Only argument marshalling happens here; every computation is a library
kernel.  torch provides the device buffers.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import qst


def init_params(d_in, h1, h2, seed):
    """Uniform He-style initial weights (bound sqrt(6/fan_in)/2), zero biases,
    as one flat FP32 array in the library's parameter order."""
    rng = np.random.default_rng(seed)

    def uni(shape, fan_in):
        b = np.sqrt(6.0 / fan_in) / 2
        return rng.uniform(-b, b, shape)
    parts = [uni((h1, d_in), d_in), np.zeros(h1), uni((h2, h1), h1), np.zeros(h2), uni((h2,), h2), np.zeros(1)]
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


@dataclass
class Pairs:
    x: object        # torch bfloat16 [N, width]
    ll: object       # torch float64 [N]
    n_chains: int
    n_slots: int


def collect_pairs(problem: qst.Problem, cfg: qst.RunConfig, pair_every, pair_chains=None) -> Pairs:
    """Run cfg (plain pCN, resumed or fresh) recording proposal pairs."""
    import torch
    pc = cfg.n_chains if pair_chains is None else pair_chains
    slots = cfg.n_steps // pair_every
    x = torch.empty((slots * pc, problem.pair_width), dtype=torch.bfloat16, device="cuda")
    ll = torch.empty(slots * pc, dtype=torch.float64, device="cuda")
    problem.run(cfg, pairs=dict(every=pair_every, chains=pc, x=x, ll=ll), stats=False)
    return Pairs(x, ll, pc, slots)


@dataclass
class TrainResult:
    mean: float
    sd: float
    losses: list = field(default_factory=list)   # (iteration, minibatch loss in standardised units)
    val_loss: float = float("nan")


def train(net: qst.Mlp, pairs: Pairs, iters, batch=1024, lr=1e-3, lr_final=1e-4, val_rows=None,
          log_every=100, seed=0):
    """Adam on consecutive minibatches of the rows in a seeded random order;
    the last `val_rows` of that order are held out.  The learning rate decays
    geometrically from lr to lr_final."""
    import torch
    n = pairs.x.shape[0]
    val_rows = val_rows if val_rows is not None else min(n // 10, 16384) // batch * batch
    n_train = (n - val_rows) // batch * batch
    if n_train < batch:
        raise ValueError("not enough pairs for one minibatch")
    y0 = torch.empty(n, dtype=torch.float32, device="cuda")
    mean, sd = qst.standardise_targets(pairs.ll, y0)
    res = TrainResult(mean, sd)
    # one fixed random order of all rows (seeded), so a minibatch mixes chains
    # and recording slots
    perm = torch.from_numpy(np.random.default_rng(seed).permutation(n).astype(np.int64)).cuda()
    xs = torch.empty_like(pairs.x)
    y = torch.empty_like(y0)
    qst.gather_rows(pairs.x, y0, perm, xs, y)
    del y0
    nb = n_train // batch
    for it in range(iters):
        rate = lr * (lr_final / lr) ** (it / max(iters - 1, 1))
        off = (it % nb) * batch
        want = (it % log_every == 0) or it == iters - 1
        loss = net.train_step(xs, y, rate, want_loss=want, rows=batch, offset=off)
        if want:
            res.losses.append((it, loss))
    if val_rows:
        # mean squared error on the held-out rows, standardised units
        _, res.val_loss = net.gradients(xs[n - val_rows:], y[n - val_rows:])
    # predictions in log-likelihood units from now on
    params = net.get_params()
    net.set_params(params, out_scale=sd, out_shift=mean)
    return res
