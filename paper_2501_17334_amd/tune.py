"""Autotuner for the chain kernel's launch shape (team size G, workgroup WG)
per qubit count.

For every compiled shape of a qubit count it runs the same synthetic problem
(Haar pure state + 10% white noise, 1024 shots per setting) for a fixed number
of chains and steps, times the launch with HIP events, and keeps the fastest
shape.  The table is written as JSON next to the library and installed in the
library through qst_set_launch_shape; `load()` installs a saved table.
"""
from __future__ import annotations

import json
import os
import sys

from . import qst, synth

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_gfx950.json")

# chains x steps timed per qubit count (enough work to fill the GPU)
WORK = {1: (65536, 400), 2: (65536, 300), 3: (65536, 100), 4: (32768, 60), 5: (4096, 20), 6: (1024, 4)}


def _problem(Q):
    rng_name = {1: "c1", 2: "c2", 4: "c3", 5: "c4"}
    if Q in rng_name:
        return synth.make_problem(rng_name[Q])
    return next(p for p in synth.mixed_batch(256) if p.n_qubits == Q)


def time_shape(Q, shape, chains, steps):
    import torch
    qst.set_launch_shape(Q, *shape)
    prob = _problem(Q)
    P = qst.Problem(Q, prob.counts)
    cfg = qst.RunConfig(n_chains=chains, n_steps=steps, seed=prob.seed, beta0=0.01, adapt_every=0)
    P.run(qst.RunConfig(n_chains=chains, n_steps=1, seed=prob.seed, beta0=0.01, adapt_every=0), stats=False)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    P.run(cfg, stats=False)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    P.close()
    return chains * steps / (ms / 1e3)


def tune(qubits=(1, 2, 3, 4, 5, 6), out=TABLE, verbose=True):
    table = {}
    for Q in qubits:
        chains, steps = WORK[Q]
        best = None
        trials = []
        for shape in qst.list_launch_shapes(Q):
            rate = time_shape(Q, shape, chains, steps)
            trials.append({"team": shape[0], "workgroup": shape[1], "chain_steps_per_s": rate})
            if verbose:
                print(f"[tune] Q={Q} G={shape[0]} WG={shape[1]}: {rate:.4g} chain-steps/s", flush=True)
            if best is None or rate > best[1]:
                best = (shape, rate)
        qst.set_launch_shape(Q, *best[0])
        table[str(Q)] = {"team": best[0][0], "workgroup": best[0][1], "chain_steps_per_s": best[1],
                         "trials": trials, "chains": chains, "steps": steps}
    if out:
        with open(out, "w") as f:
            json.dump(table, f, indent=1)
    return table


def load(path=TABLE):
    """Install a saved table (shapes that are not compiled are skipped)."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    for q, ent in table.items():
        try:
            qst.set_launch_shape(int(q), int(ent["team"]), int(ent["workgroup"]))
        except qst.QstError:
            pass
    return table


if __name__ == "__main__":
    qs = tuple(int(a) for a in sys.argv[1:]) or (1, 2, 3, 4, 5, 6)
    tune(qs)
