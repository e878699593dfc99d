"""Autotuner of the chain kernel: launch shape and contraction path.

Shapes: for every compiled (team size G, workgroup WG) of a qubit count it
runs the same synthetic problem (Haar pure state + 10% white noise, 1024
shots per setting) for a fixed number of chains and steps, times the launch
with HIP events, and keeps the fastest shape (qst_set_launch_shape).  Batch
tiles keep one team per qubit count (qst_get_batch_shape); the table records
whether it is the tuned one, since a batch problem equals its solo run bit
for bit only with the same team.

Paths: per qubit count (1..4) and precision (FP64, FP32) it times the chain
step on the Kronecker route and on the dense MFMA contraction, each with its
own launch shape, and makes the faster one what QST_PATH_AUTO takes
(qst_set_auto_path); BF16x3 exists on the dense path only.  Beside it, the
contraction alone (qst_loglik on given states, 1..5 qubits) on both paths,
so the choice can be read against the raw contraction rates.

The table is written as JSON next to the library; the binding installs it
when the library is loaded, and `load()` installs a saved table.
"""
from __future__ import annotations

import json
import os
import sys

from . import qst, synth

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_gfx950.json")

# chains x steps timed per qubit count (enough work to fill the GPU)
WORK = {1: (65536, 400), 2: (65536, 300), 3: (65536, 100), 4: (32768, 60), 5: (4096, 20), 6: (4096, 20)}


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


def time_path(Q, path, precision, chains, steps):
    """Chain-steps/s of plain pCN on `path` in `precision` (the path's own
    launch shape: the tuned one for Kronecker, 16 chains per workgroup dense)."""
    import torch
    prob = _problem(Q)
    P = qst.Problem(Q, prob.counts, precision=precision, path=path)
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


def contraction_rates(Q, n_states=None, reps=3):
    """qst_loglik on n_states given density matrices: matrices/s per (path,
    precision) -- the probability contraction and log-likelihood alone."""
    import numpy as np
    import torch
    prob = _problem(Q)
    D = 2 ** Q
    n = n_states or {1: 65536, 2: 65536, 3: 65536, 4: 65536, 5: 8192}[Q]
    rng = np.random.default_rng(5)
    base = np.stack([synth.random_density_matrix(D, rng) for _ in range(16)])
    rhos = np.ascontiguousarray(np.stack([base.real, base.imag], -1)[np.arange(n) % 16])
    dev = torch.from_numpy(rhos).cuda()
    out = torch.zeros(n, dtype=torch.float64, device="cuda")
    P = qst.Problem(Q, prob.counts)
    res = {}
    for path, prec in (("kron", "fp64"), ("kron", "fp32"), ("dense", "fp64"), ("dense", "fp32"), ("dense", "bf16x3")):
        P.loglik(dev, out, path=path, precision=prec)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            P.loglik(dev, out, path=path, precision=prec)
        b.record()
        torch.cuda.synchronize()
        res[f"{path}_{prec}"] = n / (a.elapsed_time(b) / reps / 1e3)
    P.close()
    return res


def tune_paths(qubits=(1, 2, 3, 4), verbose=True):
    """The faster path of the chain step per qubit count and precision,
    installed for QST_PATH_AUTO; returns the measured rates."""
    out = {}
    for Q in qubits:
        chains, steps = WORK[Q]
        out[str(Q)] = {}
        for prec in ("fp64", "fp32"):
            kr = time_path(Q, "kron", prec, chains, steps)
            de = time_path(Q, "dense", prec, chains, steps)
            best = "kron" if kr >= de else "dense"
            qst.set_auto_path(Q, prec, best)
            out[str(Q)][prec] = {"path": best, "kron_chain_steps_per_s": kr, "dense_chain_steps_per_s": de}
            if verbose:
                print(f"[tune] Q={Q} {prec}: kron {kr:.4g}, dense {de:.4g} chain-steps/s -> {best}", flush=True)
    return out


def tune(qubits=(1, 2, 3, 4, 5, 6), out=TABLE, verbose=True, paths=True):
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
        bteam = qst.get_batch_shape(Q)[0]
        table[str(Q)] = {"team": best[0][0], "workgroup": best[0][1], "chain_steps_per_s": best[1],
                         "trials": trials, "chains": chains, "steps": steps,
                         "batch_team": bteam, "batch_team_is_tuned_team": bteam == best[0][0]}
        if verbose and bteam != best[0][0]:
            print(f"[tune] Q={Q}: batch tiles use team {bteam}, single launches tune to {best[0][0]}; "
                  f"batch runs then differ from solo runs in summation order", flush=True)
    if paths:
        table["paths"] = tune_paths(tuple(q for q in qubits if q <= 4), verbose)
        table["contraction_states_per_s"] = {}
        for Q in (q for q in qubits if q <= 5):
            table["contraction_states_per_s"][str(Q)] = r = contraction_rates(Q)
            if verbose:
                print(f"[tune] Q={Q} contraction alone: " + ", ".join(f"{k} {v:.3g}" for k, v in r.items()),
                      flush=True)
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
        if not q.isdigit():
            continue
        try:
            qst.set_launch_shape(int(q), int(ent["team"]), int(ent["workgroup"]))
        except qst.QstError:
            pass
    for q, per in table.get("paths", {}).items():
        for prec, ent in per.items():
            qst.set_auto_path(int(q), prec, ent["path"])
    return table


if __name__ == "__main__":
    qs = tuple(int(a) for a in sys.argv[1:]) or (1, 2, 3, 4, 5, 6)
    tune(qs)
