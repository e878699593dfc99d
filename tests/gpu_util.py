"""Shared helpers of the GPU parity tests: run the HIP library and the CPU
oracle on the same problem and the same streams."""
import numpy as np
import torch

from oracle import oracle as O
from paper_2501_17334_amd import qst


def gpu_run(Q, counts, *, n_chains, n_steps, seed, beta0, thin=1, burn_in=0, adapt_every=500,
            trace=0, record_every=0, record_chains=0, precision="fp64", path="auto", problem=None,
            resume=False):
    prob = problem or qst.Problem(Q, counts, precision=precision, path=path)
    tr = rec = None
    if trace:
        tr = dict(chains=trace,
                  llprop=torch.full((trace, n_steps), float("nan"), dtype=torch.float64, device="cuda"),
                  logu=torch.zeros((trace, n_steps), dtype=torch.float64, device="cuda"),
                  accept=torch.zeros((trace, n_steps), dtype=torch.int8, device="cuda"))
    if record_every and record_chains:
        D = 2 ** Q
        rec = dict(every=record_every, chains=record_chains,
                   buf=torch.zeros((record_chains, n_steps // record_every, D, D), dtype=torch.float64,
                                   device="cuda"))
    cfg = qst.RunConfig(n_chains=n_chains, n_steps=n_steps, seed=seed, beta0=beta0, thin=thin,
                        burn_in=burn_in, adapt_every=adapt_every, resume=resume)
    stats = prob.run(cfg, trace=tr, record=rec)
    torch.cuda.synchronize()
    out = {"problem": prob, "stats": stats}
    if tr:
        out["trace_llprop"] = tr["llprop"].cpu().numpy()
        out["trace_logu"] = tr["logu"].cpu().numpy()
        out["trace_accept"] = tr["accept"].cpu().numpy()
    if rec:
        out["records"] = rec["buf"].cpu().numpy()
    return out


def oracle_run(Q, counts, *, n_chains, n_steps, seed, beta0, thin=1, burn_in=0, adapt_every=500,
               trace=0, record_every=0, record_chains=0):
    ch = O.Chains(Q, counts, O.RunParams(n_chains=n_chains, n_steps=0, seed=seed, beta0=beta0, thin=thin,
                                         burn_in=burn_in, adapt_every=adapt_every, trace_chains=trace,
                                         record_every=record_every, record_chains=record_chains))
    ll0 = ch.ll.copy()
    out = ch.run(n_steps)
    out["ll0"] = ll0
    return ch, out


def first_near_step(llprop_a, llprop_b, logu, ll0, accept, tol=1e-8):
    """Per chain, the first step at which |log u - dlogL| < tol on either side's
    log L trace (comparisons stop there)."""
    R, T = llprop_a.shape
    first = np.full(R, T)
    for r in range(R):
        ll = ll0[r]
        for t in range(T):
            d_a = llprop_a[r, t] - ll
            d_b = llprop_b[r, t] - ll
            if abs(logu[r, t] - d_a) < tol or abs(logu[r, t] - d_b) < tol:
                first[r] = t
                break
            if accept[r, t]:
                ll = llprop_b[r, t]
    return first
