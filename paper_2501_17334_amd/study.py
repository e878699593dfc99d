"""Scaling of pooled chains, after the paper's Section "Simulated Results"
(Figs. 3 and 4), on synthetic data and one GPU.

For each thinning T, R_max chains of Algorithm 2 run N T steps (N stored
samples each, no burn-in, beta starting at 0.1 with the adaptation of
Algorithm 2) in one launch.  From each run:

* the IACT tau of Eq. (IACT) from the ACF of Eq. (ACFrho) over recorded
  chains (l_max = 200, or N/4 for shorter chains), and N_eff = N R / tau;
* for R = 1, 2, 4, ..., R_max the estimate of Eq. (BME2) pooled over the
  first R chains (from each chain's own moment sums), its squared
  Frobenius error Eq. (fro) against the reference estimate at T_max and
  R_max (the paper's stand-in for the Bayesian mean), and the infidelity
  1 - F of Eq. (fid) against the same reference and against the true state;
* the wall-clock time of the launch (HIP events): on one GPU the R_max
  chains run side by side, so this is the time a single chain of the same
  length takes too (the paper's "average wall clock time").

Command line: python -m paper_2501_17334_amd.study [--qubits 1 2 3 4]
[--thinning 1 4 16 64 256 1024] [--samples 1024] [--chains 4096]
[--param gamma|bures] [--out study.json]; one JSON document on stdout (or
into --out), progress on stderr.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import qst, synth


def unpack(packed):
    """Packed real form (P[a][b] = Re rho_ab for a <= b, Im rho_ba for a > b)
    to the complex Hermitian matrix; works on [..., D, D]."""
    P = np.asarray(packed, dtype=np.float64)
    up = np.triu(P)
    im = np.swapaxes(np.tril(P, -1), -1, -2)          # Im rho_ab for a < b
    m = up + 1j * im
    return m + np.swapaxes(np.triu(m, 1), -1, -2).conj()


def _numerical_rank_clip(w):
    """Eigenvalues below the numerical-rank threshold D eps max|w| (round-off
    of a rank-deficient matrix, whose square roots would be ~1e-8) as 0."""
    tol = w.size * np.finfo(np.float64).eps * max(float(np.max(np.abs(w))), 1e-300)
    return np.where(w > tol, w, 0.0)


def _psd_sqrt(rho):
    w, V = np.linalg.eigh((rho + rho.conj().T) / 2)
    return (V * np.sqrt(_numerical_rank_clip(w))) @ V.conj().T


def fidelity(rho, sigma):
    """Eq. (fid): (Tr sqrt(sqrt(rho) sigma sqrt(rho)))^2 for density matrices,
    by eigendecompositions of Hermitian matrices."""
    s = _psd_sqrt(rho)
    m = s @ sigma @ s
    w = np.linalg.eigvalsh((m + m.conj().T) / 2)
    return float(np.sum(np.sqrt(_numerical_rank_clip(w))) ** 2)


def chain_counts(R_max):
    out, r = [], 1
    while r < R_max:
        out.append(r)
        r *= 2
    return out + [R_max]


def run_thinning(P, cfg_kw, T, N, R_max, record_chains, torch):
    """One launch of R_max chains with thinning T; per-chain sums, tau, time."""
    D = P.D
    cfg = qst.RunConfig(n_chains=R_max, n_steps=N * T, thin=T, burn_in=0, **cfg_kw)
    rec = torch.zeros((record_chains, N, D, D), dtype=torch.float64, device="cuda")
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    P.run(cfg, record=dict(every=T, chains=record_chains, buf=rec), stats=False)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    s1, _ = P.moments()
    nst = P.state()[3]
    tau = qst.iact(qst.acf(rec, l_max=min(200, max(1, N // 4))))   # the paper: l_max = 200 at N = 1024
    return {"ms": ms, "s1": s1, "n_stored": nst, "tau": tau}


def study(Q, counts, truth, *, T_list, N, R_max, record_chains=64, seed=1, param="gamma", log=None):
    import torch
    P = qst.Problem(Q, counts, param=param)
    cfg_kw = dict(seed=seed, beta0=0.1, adapt_every=500)
    runs = {}
    for T in T_list:
        runs[T] = run_thinning(P, cfg_kw, T, N, R_max, record_chains, torch)
        if log:
            log(f"[study] Q={Q} {param} T={T}: {runs[T]['ms']:.0f} ms, tau {runs[T]['tau']:.2f}")
    P.close()
    Rs = chain_counts(R_max)
    ref_run = runs[max(T_list)]
    ref = unpack(ref_run["s1"].sum(0) / ref_run["n_stored"].sum())
    out = {"Q": Q, "param": param, "N": N, "R_max": R_max, "T": list(T_list), "R": Rs,
           "reference_fidelity_to_truth": fidelity(truth, ref), "runs": []}
    for T in T_list:
        r = runs[T]
        cs1 = np.cumsum(r["s1"], axis=0)
        cn = np.cumsum(r["n_stored"])
        eps2, inf_ref, inf_truth = [], [], []
        for R in Rs:
            est = unpack(cs1[R - 1] / cn[R - 1])
            eps2.append(float(np.sum(np.abs(est - ref) ** 2)))
            inf_ref.append(1.0 - fidelity(ref, est))
            inf_truth.append(1.0 - fidelity(truth, est))
        out["runs"].append({"T": T, "ms": r["ms"], "tau": r["tau"],
                            "n_eff": [N * R / r["tau"] for R in Rs], "eps_f2": eps2,
                            "infidelity_to_reference": inf_ref, "infidelity_to_truth": inf_truth})
    # Fig. 4(b): the least time at which R_max chains reach F > 1 - 10^-k
    # against the reference (no entry if no run does)
    thresholds = {}
    for k in range(1, 6):
        hit = [run["ms"] for run in out["runs"] if run["infidelity_to_reference"][-1] < 10.0 ** -k]
        thresholds[str(k)] = min(hit) if hit else None
    out["ms_to_fidelity_1_minus_10_to_minus_k"] = thresholds
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--qubits", type=int, nargs="+", default=[1, 2, 3, 4])
    ap.add_argument("--thinning", type=int, nargs="+", default=[1, 4, 16, 64, 256, 1024])
    ap.add_argument("--samples", type=int, default=1024)
    ap.add_argument("--chains", type=int, default=4096)
    ap.add_argument("--record-chains", type=int, default=64)
    ap.add_argument("--param", default="gamma", choices=["gamma", "bures"])
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    res = []
    for Q in a.qubits:
        prob = synth.make_problem(f"w_{Q}")
        res.append(study(Q, prob.counts, prob.truth.density_matrix(), T_list=sorted(a.thinning), N=a.samples,
                         R_max=a.chains, record_chains=min(a.record_chains, a.chains), seed=prob.seed,
                         param=a.param, log=log))
    doc = {"what": "pooled-chain scaling after the paper's Figs. 3-4: W states with 10% white noise, "
                   "25 * 2^Q shots per Pauli setting", "studies": res}
    text = json.dumps(doc)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    print(text, flush=True)


if __name__ == "__main__":
    main()
