#!/usr/bin/env python3
"""Throughput of the pooled pCN tomography sampler on one MI355X.

One bench step = the whole hot path on the 4-qubit workload: initialise
65536 chains (step 0), run 10^4 pCN steps of Algorithm 2 on each (proposal,
rho, Pauli probabilities, FP64 log-likelihood, accept, adaptation, moments,
recording of 256 chains every 4 steps) in one persistent launch, then pool
(Eq. (BME2)).  Inputs are synthetic (seeded multinomial counts of
0.95|GHZ_4><GHZ_4| + 0.05 I/16, 1024 shots x 81 settings) and resident in HBM.

Prints one JSON line: chain-steps/s as `value`, pooled ESS/s beside it, the
roofline of the chain kernel and the CPU oracle's rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X FP64 vector (published)


def algorithmic_flops_per_chain_step(Q):
    """The algorithmic work of one chain-step that the roofline prices: the
    Kronecker-factored contraction (Q per-qubit 4 -> 6 maps on the Hermitian
    tensor, sum_q 8 6^q 4^(Q-q) flop: 24,960 at 4 qubits) plus the rho build
    (a Hermitian rank-D complex update, 4 D^3 flop: 16,384 at 4 qubits);
    41,344 flop at 4 qubits.  Normals and logarithms are counts, not flops."""
    D = 2 ** Q
    contraction = sum(8 * 6 ** q * 4 ** (Q - q) for q in range(1, Q + 1))
    return contraction + 4 * D ** 3


def flops_per_chain_step(Q, stored_fraction):
    """Every FP64 flop of the method's arithmetic in one chain-step (proposal,
    weights, rho, contraction, count-weighted log sum, moments): reported
    beside the roofline, which prices the algorithmic work only."""
    D = 2 ** Q
    d = 2 * D * D + D
    KD = 6 ** Q
    proposal = 2 * d                       # a*y + beta*eta
    weights = 4 * D * D + 3 * D            # column norms, v^2 / sum / |z|^2
    rho = 4 * D ** 3                       # Hermitian rank-D update (complex)
    contraction = sum(8 * 6 ** q * 4 ** (Q - q) for q in range(1, Q + 1))  # per-qubit 4->6 maps
    loglik = 2 * KD                        # c * log p, summed
    moments = 3 * D * D * stored_fraction  # S1 += rho, S2 += rho^2
    return proposal + weights + rho + contraction + loglik + moments


def flops_per_chain_step_bures(Q, stored_fraction):
    """Algorithmic FP64 flops of one chain-step with Algorithm 1 (the Bures
    draw): the same contraction, likelihood and moments, with the proposal
    over 4D^2 parameters and rho from Gram-Schmidt of H, W = (U + I) G and the
    Gram product of W."""
    D = 2 ** Q
    d = 4 * D * D
    KD = 6 ** Q
    proposal = 2 * d
    qr = 6 * D * D + 8 * D * D * (D - 1)   # column norms and scaling; c = u^dag a and a -= c u for j > k
    w = 8 * D ** 3                         # (U + I) G, complex
    trace = 4 * D * D
    rho = 4 * D ** 3 + D * D               # Hermitian Gram product of W, scaled
    contraction = sum(8 * 6 ** q * 4 ** (Q - q) for q in range(1, Q + 1))
    loglik = 2 * KD
    moments = 3 * D * D * stored_fraction
    return proposal + qr + w + trace + rho + contraction + loglik + moments


def flops_per_chain_step_dense(Q, stored_fraction, rows=None):
    """Algorithmic flops of one chain-step on the dense path: the default
    parameterisation's proposal, weights, rho and moments, the contraction
    p = M vec rho as a dense product over the D^2 packed reals of rho for each
    of the rows of M (K D Pauli projectors, or the user's POVM elements), and
    the count-weighted log sum.  Returns (total, contraction)."""
    D = 2 ** Q
    rows = 6 ** Q if rows is None else rows
    d = 2 * D * D + D
    contraction = 2 * rows * D * D
    rest = 2 * d + 4 * D * D + 3 * D + 4 * D ** 3 + 2 * rows + 3 * D * D * stored_fraction
    return contraction + rest, contraction


MFMA_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}


def dense_rate_entry(what, R, steps, ms, Q, prec, rows=None):
    """Rate of a dense-path run with the achieved rate of its contraction
    flops against the MFMA peak of the contraction's precision (BF16x3: the
    algorithmic flops of the product, against the BF16 peak)."""
    total, con = flops_per_chain_step_dense(Q, 1.0, rows)
    rate = R * steps / (ms / 1e3)
    return {"what": what, "chain_steps_per_s": rate, "ms": ms, "flop_per_chain_step": total,
            "contraction_flop_per_chain_step": con, "contraction_tflops": rate * con / 1e12,
            "mfma_peak_tflops": MFMA_PEAK_TFLOPS[prec], "frac_mfma_peak": rate * con / 1e12 / MFMA_PEAK_TFLOPS[prec]}


def kernel_source_hash():
    """Hash of the code the chain kernel is compiled from (its device code:
    the step, the random numbers, the fast math), comments and blank space
    removed, so that only a change of code invalidates measured counters."""
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2501_17334_amd", "csrc")
    for name in ("chain_kernel.hpp", "fastmath.hpp", "rng.hpp"):
        with open(os.path.join(csrc, name)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(name.encode())
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_counter(kernel_hash, key, field):
    """A figure from the committed rocprofv3 --pmc summaries
    (profiles/traffic.json), if they were taken on the current kernel
    sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    ent = data.get(key)
    if not ent or ent.get("kernel_source_hash") != kernel_hash:
        return None
    return ent.get(field)


def measured_traffic(kernel_hash, key):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated)."""
    return measured_counter(kernel_hash, key, "bytes_per_launch")


def valu_issue(kernel_hash, key, chain_steps_per_s):
    """Vector-instruction issue of the chain launch: the profiled
    SQ_INSTS_VALU per chain-step (one count per wavefront instruction) times
    the live chain-step rate, against the issue peak of wave64 VALU work,
    one wavefront instruction per 4 cycles on each 16-lane SIMD (256 CUs x 4
    SIMDs x 2.4 GHz / 4); None without a profile of the current sources."""
    per_step = measured_counter(kernel_hash, key + "_valu", "valu_instr_per_chain_step")
    if per_step is None:
        return None
    peak = 256 * 4 * 2.4e9 / 4
    achieved = per_step * chain_steps_per_s
    return {"instr_per_chain_step": per_step, "achieved_per_s": achieved, "peak_per_s": peak,
            "frac": achieved / peak, "source": measured_counter(kernel_hash, key + "_valu", "summary")}


def dense_gemm_rates(qst, synth, torch, prob, n_states=65536, reps=5):
    """Throughput of the dense contraction kernel alone (qst_loglik, dense
    path) on n_states density matrices, per precision: algorithmic GEMM
    flops 2 KD D^2 per state over the kernel time, against the MFMA peak of
    the operand type (FP64 78.6, FP32 157.3, BF16 2500 TFLOP/s; BF16x3
    counts its three products)."""
    import numpy as np
    Q, D = prob.n_qubits, 2 ** prob.n_qubits
    rng = np.random.default_rng(5)
    base = np.stack([synth.random_density_matrix(D, rng) for _ in range(64)])
    rhos = np.ascontiguousarray(np.stack([base.real, base.imag], -1)[np.arange(n_states) % 64])
    dev = torch.from_numpy(rhos).cuda()
    out = torch.zeros(n_states, dtype=torch.float64, device="cuda")
    flop = 2.0 * (6 ** Q) * D * D * n_states
    res = {}
    for prec, peak, mult in (("fp64", 78.6, 1), ("fp32", 157.3, 1), ("bf16x3", 2500.0, 3)):
        P = qst.Problem(Q, prob.counts, precision=prec, path="dense")
        P.loglik(dev, out, path="dense", precision=prec)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            P.loglik(dev, out, path="dense", precision=prec)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        tf = mult * flop / (ms / 1e3) / 1e12
        res[prec] = {"ms": ms, "tflops": tf, "peak": peak, "frac": tf / peak, "states": n_states}
        P.close()
    return res


def chosen_forms(qst, torch, np, prob, cfg, record, plain_pool, plain_ms, plain_tau, plain_ess_between,
                 dense_steps=1000):
    """The production forms on the same workload, same seeds and the pilot
    beta: the mixed-precision Kronecker form over the full run (rate, ESS
    from its own records, pooled-mean difference against the plain FP64 run
    in units of the plain run's between-chain standard error), and the dense
    MFMA contraction inside the chain kernel in each precision over a short
    run (rate only)."""
    import dataclasses
    out = {}
    Q, R, NT = prob.n_qubits, cfg.n_chains, cfg.n_steps
    se_f = float(np.sqrt(np.sum(plain_pool["se_re"] ** 2 + plain_pool["se_im"] ** 2)))

    def timed(P, c, rec):
        P.run(dataclasses.replace(c, n_chains=256, n_steps=10), stats=False)     # module load, attributes
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        P.run(c, record=rec, stats=False)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    P = qst.Problem(Q, prob.counts, precision="fp32", path="kron")
    rec_buf = record["buf"]
    ms = timed(P, cfg, record)
    pool = P.pool()
    every = record["every"]
    first = (cfg.burn_in + every - 1) // every
    n_rec = NT // every - first
    c = qst.acf(rec_buf[:, first:].contiguous(), l_max=min(200, n_rec - 1))
    tau = qst.iact(c)
    var = np.concatenate([(pool["second_re"] - pool["mean"].real ** 2).ravel(),
                          (pool["second_im"] - pool["mean"].imag ** 2).ravel()])
    se2 = np.concatenate([pool["se_re"].ravel() ** 2, pool["se_im"].ravel() ** 2])
    ess_between = float(np.sum(var) / np.sum(se2))
    diff = float(np.sqrt(np.sum(np.abs(pool["mean"] - plain_pool["mean"]) ** 2)))
    out["kron_fp32"] = {
        "what": "Pauli coefficients, per-setting Walsh-Hadamard transforms and log2 p in FP32, "
                "count-weighted sum and acceptance in FP64; full run, same seeds and beta",
        "chain_steps_per_s": R * NT / (ms / 1e3), "ms": ms,
        "speedup_vs_plain_fp64": plain_ms / ms,
        "tau": tau, "tau_plain_fp64": plain_tau,
        "ess_per_s": n_rec * R / tau / (ms / 1e3),
        "between_chain_ess_per_s": ess_between / (ms / 1e3),
        "between_chain_ess_per_s_plain_fp64": plain_ess_between / (plain_ms / 1e3),
        "mean_diff_frobenius_vs_plain_fp64": diff, "plain_fp64_se_frobenius": se_f,
        "mean_diff_in_se": diff / se_f,
    }
    P.close()
    if Q <= 4:
        for prec in ("fp64", "fp32", "bf16x3"):
            P = qst.Problem(Q, prob.counts, precision=prec, path="dense")
            c2 = dataclasses.replace(cfg, n_steps=dense_steps, burn_in=0)
            ms = timed(P, c2, None)
            out[f"dense_{prec}"] = dense_rate_entry(f"dense MFMA contraction in the chain kernel ({prec}), "
                                                    f"{dense_steps}-step run, moments every step", R, dense_steps,
                                                    ms, Q, prec)
            P.close()
    return out


def bures_form(qst, torch, np, prob, cfg, plain_pool):
    """The paper's own parameterisation (Algorithm 1, the Bures draw) on the
    same workload: its own pilot beta, the full run, its rate and the
    achieved FP64 rate of its algorithmic flops, and the Frobenius distance
    of its pooled mean to the true state next to the plain run's.  With
    4D^2 parameters the pilot beta is about half the plain one and the
    chains are still travelling towards the posterior after 10^4 steps, so
    no ESS is reported for them."""
    import dataclasses
    Q, R, NT = prob.n_qubits, cfg.n_chains, cfg.n_steps
    P = qst.Problem(Q, prob.counts, param="bures")
    beta, pst = pilot_beta(qst, P, prob.seed)
    c = dataclasses.replace(cfg, beta0=beta)
    P.run(dataclasses.replace(c, n_chains=256, n_steps=10), stats=False)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    P.run(c, stats=False)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    pool = P.pool()
    truth = prob.truth.density_matrix()
    flop = flops_per_chain_step_bures(Q, (NT - cfg.burn_in) / NT)
    tflops = flop * R * NT / (ms / 1e3) / 1e12
    P.close()
    return {"what": "Algorithm 1 (Bures draw, 4D^2 parameters): Gram-Schmidt U = Q Lambda, W = (U + I) G, "
                    "rho = W W^dag / Tr, FP64, same workload and seeds, own pilot beta",
            "beta0_from_pilot": beta, "pilot_acceptance": pst["accepted"] / pst["proposed"],
            "chain_steps_per_s": R * NT / (ms / 1e3), "ms": ms,
            "flop_per_chain_step": flop, "achieved_tflops": tflops, "frac_fp64_peak": tflops / PEAK_FP64_TFLOPS,
            "mean_error_to_truth_frobenius": float(np.sqrt(np.sum(np.abs(pool["mean"] - truth) ** 2))),
            "plain_mean_error_to_truth_frobenius": float(np.sqrt(np.sum(np.abs(plain_pool["mean"] - truth) ** 2)))}


def option_rates(qst, synth, torch, prob, cfg, steps=1000):
    """Rates of the other options on the 4-qubit chain count, short runs: the
    default form with Dirichlet(1) weights (Gamma quantiles by Newton steps),
    and 81 random measurement bases given as POVM elements (dense path)."""
    import dataclasses
    R = cfg.n_chains
    c = dataclasses.replace(cfg, n_steps=steps, burn_in=0)
    out = {}

    def timed(P):
        P.run(dataclasses.replace(c, n_chains=256, n_steps=10), stats=False)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        P.run(c, stats=False)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    P = qst.Problem(prob.n_qubits, prob.counts, param="dirichlet", alpha=1.0)
    ms = timed(P)
    out["dirichlet_alpha1"] = {"what": "Dirichlet(1) weights, FP64 Kronecker route, rate only",
                               "chain_steps_per_s": R * steps / (ms / 1e3), "ms": ms}
    P.close()
    bp = synth.random_bases_problem(prob.n_qubits)
    for prec in ("fp64", "fp32"):
        P = qst.Problem(prob.n_qubits, bp.counts, precision=prec, povm=bp.povm)
        ms = timed(P)
        out[f"povm_random_bases_{prec}"] = dense_rate_entry(
            f"81 Haar-random bases as POVM elements, dense MFMA path ({prec}), {steps}-step run, moments every step",
            R, steps, ms, prob.n_qubits, prec, rows=bp.povm.shape[0])
        P.close()
    return out


def delayed_acceptance(qst, surrogate, synth, torch, np, name="c4", warm=4000, pair_steps=2000, pair_every=20,
                       iters=4000, steps=1000, skill_chains=64, skill_steps=300):
    """Delayed acceptance with the learned surrogate on its own workload (the
    5-qubit problem, 16384 chains): pilot beta, warm-up, training pairs from
    the chains, training on the GPU, then the same resumed state run plain
    and with the surrogate.  Also the surrogate's skill where the first stage
    needs it: predicted against exact log-likelihood differences of
    consecutive pCN proposals."""
    prob = synth.make_problem(name)
    Q, R = prob.n_qubits, prob.n_chains

    def start():
        P = qst.Problem(Q, prob.counts)
        P.run(qst.RunConfig(n_chains=256, n_steps=4000, seed=prob.seed + 99, beta0=0.1, adapt_every=100),
              stats=False)
        beta = float(np.median(P.state()[2]))
        P.run(qst.RunConfig(n_chains=R, n_steps=warm, seed=prob.seed, beta0=beta, adapt_every=500), stats=False)
        return P, beta

    A, beta = start()
    pcfg = qst.RunConfig(n_chains=R, n_steps=pair_steps, seed=prob.seed, beta0=beta, adapt_every=500, resume=True)
    pairs = surrogate.collect_pairs(A, pcfg, pair_every=pair_every)
    net = qst.Mlp(A.pair_width, 512, 512)
    net.set_params(surrogate.init_params(A.pair_width, 512, 512, seed=1))
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    tr = surrogate.train(net, pairs, iters, batch=1024, lr=1e-3, lr_final=5e-5)
    b.record()
    torch.cuda.synchronize()
    train_ms = a.elapsed_time(b)
    n_pairs = int(pairs.x.shape[0])
    del pairs
    torch.cuda.empty_cache()
    B, _ = start()
    B.run(pcfg, stats=False)
    cfg = qst.RunConfig(n_chains=R, n_steps=steps, seed=prob.seed, beta0=beta, adapt_every=500, resume=True)

    def timed(P, **kw):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        st = P.run(cfg, stats=True, **kw)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b), st

    ms_plain, st_plain = timed(B)
    ms_da, st_da = timed(A, surrogate=net.surrogate())
    # skill on consecutive proposals of the plain chains
    C, T = skill_chains, skill_steps
    x = torch.empty((T * C, B.pair_width), dtype=torch.bfloat16, device="cuda")
    ll = torch.empty(T * C, dtype=torch.float64, device="cuda")
    trc = dict(chains=C, llprop=torch.zeros((C, T), dtype=torch.float64, device="cuda"),
               logu=torch.zeros((C, T), dtype=torch.float64, device="cuda"),
               accept=torch.zeros((C, T), dtype=torch.int8, device="cuda"))
    x0, l0, _, _ = B.state()
    B.run(qst.RunConfig(n_chains=R, n_steps=T, seed=prob.seed + 1, beta0=beta, adapt_every=500, resume=True),
          trace=trc, pairs=dict(every=1, chains=C, x=x, ll=ll), stats=False)
    s_prop = net.predict(x).double().cpu().numpy().reshape(T, C)
    l_prop = ll.cpu().numpy().reshape(T, C)
    acc = trc["accept"].cpu().numpy()
    xs0 = torch.from_numpy(np.pad(x0[:C], ((0, 0), (0, B.pair_width - B.d)))).cuda()
    s_cur = net.predict(xs0).double().cpu().numpy()
    l_cur = l0[:C].copy()
    dS, dL = [], []
    for t in range(T):
        dS.append(s_prop[t] - s_cur)
        dL.append(l_prop[t] - l_cur)
        s_cur = np.where(acc[:, t] == 1, s_prop[t], s_cur)
        l_cur = np.where(acc[:, t] == 1, l_prop[t], l_cur)
    dS, dL = np.concatenate(dS), np.concatenate(dL)
    ok = np.isfinite(dL)
    dS, dL = dS[ok], dL[ok]
    rate_plain = R * steps / (ms_plain / 1e3)
    rate_da = R * steps / (ms_da / 1e3)
    acc_plain = st_plain["accepted"] / st_plain["proposed"]
    acc_da = st_da["accepted"] / st_da["proposed"]
    A.close()
    B.close()
    net.close()
    return {
        "workload": f"{name}: {Q}-qubit, {R} chains; pilot beta {beta:.4g}; warm-up {warm} steps; "
                    f"{n_pairs} training pairs (every {pair_every} steps over {pair_steps}); then {steps} steps "
                    f"plain and delayed from the same state",
        "network": f"{B.pair_width}->512->512->1 GELU, BF16 products, FP32 accumulation, Adam {iters} iterations",
        "train_ms": train_ms, "val_mse_standardised": tr.val_loss, "target_sd": tr.sd,
        "plain": {"chain_steps_per_s": rate_plain, "accept": acc_plain},
        "delayed": {"chain_steps_per_s": rate_da, "accept": acc_da,
                    "stage1_pass": st_da["stage1_passed"] / st_da["proposed"]},
        "skill": {"corr_dsurrogate_dloglik": float(np.corrcoef(dS, dL)[0, 1]),
                  "rms_dloglik": float(np.sqrt(np.mean(dL ** 2))),
                  "rms_error": float(np.sqrt(np.mean((dS - dL) ** 2)))},
        # accepted moves per second: the chains are the same method, so this is
        # the ratio of their sampling efficiency at equal step size
        "gain_accepted_moves_per_s": (rate_da * acc_da) / (rate_plain * acc_plain),
        "gain_chain_steps_per_s": rate_da / rate_plain,
    }


def uneven_batch(qst, synth, torch, np, steps=200, full_steps=2000):
    """The 256-problem batch of 1..6 qubits (256..4096 chains each) in its
    work-queue launches, against the same problems launched one after
    another with their tuned shapes; both from step 0, the same streams,
    FP64, `steps` steps.  Also per qubit count: the problems of that size
    batched against solo; the whole batch in the FP32 Kronecker form; and the
    batch over the workload's full 2000 steps in both precisions."""
    probs = synth.mixed_batch(256)

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    def compare(ps, precision="fp64"):
        cfgs = [qst.RunConfig(n_chains=p.n_chains, n_steps=steps, seed=p.seed, beta0=0.05, adapt_every=0)
                for p in ps]
        handles = [qst.Problem(p.n_qubits, p.counts, precision=precision, path="kron") for p in ps]
        work = sum(c.n_chains for c in cfgs) * steps
        if len(handles) > 1:
            qst.run_batch(handles, cfgs, stats=False)          # module load, buffers
        for h, c in zip(handles, cfgs):
            h.run(c, stats=False)
        torch.cuda.synchronize()
        ms_b = timed(lambda: qst.run_batch(handles, cfgs, stats=False)) if len(handles) > 1 else float("nan")
        ms_s = timed(lambda: [h.run(c, stats=False) for h, c in zip(handles, cfgs)])
        for h in handles:
            h.close()
        return {"problems": len(ps), "chain_steps": work, "batch_ms": ms_b, "solo_ms": ms_s,
                "batch_chain_steps_per_s": work / (ms_b / 1e3), "solo_chain_steps_per_s": work / (ms_s / 1e3),
                "speedup_vs_solo_launches": ms_s / ms_b}

    out = {"workload": f"256 problems of 1..6 qubits, 256..4096 chains each, {steps} steps from step 0, "
                       f"FP64 Kronecker route; the batch call vs one launch per problem (tuned shapes); "
                       f"and the batch over {full_steps} steps (M_A = 500)"}
    out.update(compare(probs))
    out["per_qubit_count"] = {str(q): compare([p for p in probs if p.n_qubits == q]) for q in range(1, 7)}
    # forms (1) and (2) together: the same batch with every problem in the FP32 Kronecker form
    f32 = compare(probs, precision="fp32")
    out["fp32_form"] = {k: f32[k] for k in ("batch_ms", "solo_ms", "batch_chain_steps_per_s",
                                            "solo_chain_steps_per_s", "speedup_vs_solo_launches")}
    out["fp32_form"]["batch_speedup_vs_fp64_batch"] = out["batch_ms"] / f32["batch_ms"]
    full = {}
    for precision in ("fp64", "fp32"):
        cfgs = [qst.RunConfig(n_chains=p.n_chains, n_steps=full_steps, seed=p.seed, beta0=0.05, adapt_every=500)
                for p in probs]
        handles = [qst.Problem(p.n_qubits, p.counts, precision=precision, path="kron") for p in probs]
        qst.run_batch(handles, [qst.RunConfig(n_chains=c.n_chains, n_steps=2, seed=c.seed) for c in cfgs],
                      stats=False)
        work = sum(c.n_chains for c in cfgs) * full_steps
        ms = timed(lambda: qst.run_batch(handles, cfgs, stats=False))
        full[precision] = {"ms": ms, "chain_steps": work, "chain_steps_per_s": work / (ms / 1e3)}
        for h in handles:
            h.close()
    full["fp32_speedup"] = full["fp64"]["ms"] / full["fp32"]["ms"]
    out[f"full_{full_steps}_steps"] = full
    return out


def pilot_beta(qst, P, seed, n_chains=256, n_steps=6000):
    """Algorithm 2's own adaptation (every 100 steps here) run on a pilot set
    of chains; the median final beta starts the measured run."""
    import numpy as np
    st = P.run(qst.RunConfig(n_chains=n_chains, n_steps=n_steps, seed=seed + 7919, beta0=0.1,
                             adapt_every=100), stats=True)
    _, _, beta, _ = P.state()
    return float(np.median(beta)), st


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, target_s, ess_per_chain_step=None, parity_runs=True):
    """The FP64 oracle on this host's cores, on a bounded sample of the same
    workload: 16 x threads chains from step 0, steps sized for ~target_s;
    then the same on one thread (a shorter sample), and the full 1- and
    2-qubit parity runs (64 x 2000 and 4096 x 10^4 chain-steps).  The
    oracle's ESS/s is its rate times the ESS per chain-step of the GPU run
    of the same algorithm (the chains are the same up to rounding)."""
    from oracle import oracle as O
    from paper_2501_17334_amd import synth
    threads = O.num_threads()

    def rate_on(p, R, seconds, beta0, adapt_every=500):
        ch = O.Chains(p.n_qubits, p.counts, O.RunParams(n_chains=R, n_steps=0, seed=p.seed, beta0=beta0,
                                                       adapt_every=adapt_every))
        t0 = time.perf_counter()
        ch.run(2)
        rate = 2 * R / (time.perf_counter() - t0)
        steps = max(4, int(seconds * rate / R))
        t0 = time.perf_counter()
        ch.run(steps)
        dt = time.perf_counter() - t0
        return R * steps / dt, steps, dt

    R = 16 * threads
    value, steps, dt = rate_on(prob, R, target_s, 0.01)
    O.set_num_threads(1)
    try:
        one, steps1, dt1 = rate_on(prob, 4, target_s / 4, 0.01)
    finally:
        O.set_num_threads(threads)
    out = {"value": value, "unit": "chain-steps/s", "cores": threads, "kind": "oracle",
           "sample": f"{R} chains x {steps} pCN steps of the {prob.n_qubits}-qubit workload (steps 3..{steps + 2}), "
                     f"{dt:.1f} s of FP64 CPU work on {threads} threads",
           "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
           "one_core": {"value": one, "unit": "chain-steps/s",
                        "sample": f"4 chains x {steps1} steps on one thread, {dt1:.1f} s"}}
    if ess_per_chain_step:
        out["ess_per_s"] = value * ess_per_chain_step
        out["ess_per_s_note"] = "oracle chain-steps/s x the GPU run's ESS per chain-step (same algorithm)"
    if parity_runs:
        runs = {}
        for name in ("c1", "c2"):
            p = synth.make_problem(name)
            ch = O.Chains(p.n_qubits, p.counts, O.RunParams(n_chains=p.n_chains, n_steps=0, seed=p.seed,
                                                           beta0=p.extra.get("beta0", 0.05), adapt_every=500))
            t0 = time.perf_counter()
            ch.run(p.n_steps)
            dt = time.perf_counter() - t0
            runs[name] = {"chains": p.n_chains, "steps": p.n_steps, "seconds": dt,
                          "chain_steps_per_s": p.n_chains * p.n_steps / dt}
        out["parity_runs_full"] = runs
    return out


def calibrate_copy(torch, mib, reps=3):
    """A plain device-to-device copy of a known size: run under
    `rocprofv3 --pmc FETCH_SIZE` (then `WRITE_SIZE`), each copy dispatch reads
    and writes mib MiB, and the ratio of a counter to that figure scales the
    same counter of another kernel on the same machine."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for r in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        print(f"copy {r}: {n * 8} bytes read + {n * 8} written in {ms:.3f} ms ({2 * n * 8 / ms / 1e6:.1f} GB/s)",
              flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--chains", type=int, default=None)
    ap.add_argument("--nsteps", type=int, default=10000)
    ap.add_argument("--burn-in", type=int, default=5000)
    ap.add_argument("--record-every", type=int, default=4)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (the known-size "
                         "dispatch that scales rocprofv3's FETCH_SIZE/WRITE_SIZE counters) and exit")
    ap.add_argument("--path", default="auto")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dense-gemm", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-delayed", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported. The chains need no "
              f"communication: each GPU would run its own chain range (qst_run_desc.chain_offset) and the "
              f"moment totals would be summed once at the end.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        calibrate_copy(torch, args.calibrate_copy)
        return

    from paper_2501_17334_amd import qst, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prob = synth.make_problem(args.config, n_chains=args.chains)
    Q, D = prob.n_qubits, 2 ** prob.n_qubits
    R, NT, burn = prob.n_chains, args.nsteps, args.burn_in
    P = qst.Problem(Q, prob.counts, precision=args.precision, path=args.path)

    print(f"[bench] workload {args.config}: Q={Q} chains={R} steps={NT}; pilot", file=sys.stderr, flush=True)
    beta, pst = pilot_beta(qst, P, prob.seed)
    print(f"[bench] pilot beta={beta:.5g} (acceptance {pst['accepted'] / pst['proposed']:.3f})",
          file=sys.stderr, flush=True)

    # 1250 recorded samples per chain after the burn-in (every 4 steps of the
    # last 5000): Eq. (IACT) needs N well above tau for a trustworthy sum
    rec_every, rec_chains = args.record_every, min(256, R)
    rec = torch.zeros((rec_chains, NT // rec_every, D, D), dtype=torch.float64, device=dev)
    cfg = qst.RunConfig(n_chains=R, n_steps=NT, seed=prob.seed, beta0=beta, thin=1, burn_in=burn,
                        adapt_every=500)
    record = dict(every=rec_every, chains=rec_chains, buf=rec)

    def step():
        P.run(cfg, record=record, stats=False)

    for w in range(args.warmup):
        step()
        P.pool()
        torch.cuda.synchronize()
        print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    k_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start.record(stream)
    pool = None
    for k in range(args.steps):
        k_ev[k][0].record(stream)
        step()
        k_ev[k][1].record(stream)
        pool = P.pool()          # waits for the run
        print(f"[bench] step {k + 1}/{args.steps} done", file=sys.stderr, flush=True)
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_total = t_start.elapsed_time(t_end)
    ms_step = ms_total / args.steps
    ms_kernel = float(np.mean([a.elapsed_time(b) for a, b in k_ev]))
    chain_steps = R * NT
    value = chain_steps / (ms_step / 1e3)

    # pooled ESS two ways: N_eff = N R / tau with tau from Eq. (IACT) on the
    # recorded chains after the burn-in, and the between-chain ESS
    # tr Var_post / SE^2 of the independent chains
    first = (burn + rec_every - 1) // rec_every
    n_rec = NT // rec_every - first
    l_max = min(200, n_rec - 1)
    c = qst.acf(rec[:, first:].contiguous(), l_max=l_max)
    tau = qst.iact(c)
    n_eff_iact = n_rec * R / tau
    var = np.concatenate([(pool["second_re"] - pool["mean"].real ** 2).ravel(),
                          (pool["second_im"] - pool["mean"].imag ** 2).ravel()])
    se2 = np.concatenate([pool["se_re"].ravel() ** 2, pool["se_im"].ravel() ** 2])
    ess_between = float(np.sum(var) / np.sum(se2))
    # Eq. (IACT) truncated at l_max is only trustworthy when the ACF has died
    # out there: flag a tail still above 0.05, a sum pulled down by negative
    # values (each chain is centred on its own mean, which biases every c[l]
    # low by about tau/N), and disagreement with the between-chain ESS; the
    # headline ESS is the smaller of the two estimates
    ratio = n_eff_iact / ess_between
    ess_flags = {"tail_above_0.05": bool(c[-1] > 0.05), "acf_below_-0.05": bool(np.min(c) < -0.05),
                 "iact_vs_between_ratio_beyond_1.5": bool(ratio > 1.5 or ratio < 1 / 1.5)}
    n_eff = min(n_eff_iact, ess_between)

    stored_fraction = (NT - burn) / NT
    flop_all = flops_per_chain_step(Q, stored_fraction)
    flop = algorithmic_flops_per_chain_step(Q)
    achieved = flop * chain_steps / (ms_kernel / 1e3) / 1e12
    khash = kernel_source_hash()
    traffic = measured_traffic(khash, f"chain_kernel_q{Q}_{args.config}")

    out = {
        "metric": "pooled ESS/s and pCN chain-steps/s, 4-qubit QST, plain FP64 vs chosen form",
        "value": value,
        "unit": "chain-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.config}: {Q}-qubit Pauli tomography ({3 ** Q} settings x {D} outcomes, "
                        f"{prob.shots} shots/setting, seeded counts); {R} chains x {NT} pCN steps, "
                        f"burn-in {burn}, moments every step, {rec_chains} chains recorded every "
                        f"{rec_every} steps",
            "n_chains": R, "n_steps": NT, "path": args.path, "precision": args.precision,
            "beta0_from_pilot": beta,
        },
        "ess_per_s": n_eff / (ms_step / 1e3),
        "ess": {"headline": "min(IACT ESS, between-chain ESS)", "n_eff": n_eff,
                "iact_n_eff": n_eff_iact, "iact_ess_per_s": n_eff_iact / (ms_step / 1e3),
                "tau": tau, "tau_steps": tau * rec_every, "tau_spacing_steps": rec_every,
                "records_per_chain": n_rec, "recorded_chains": rec_chains, "l_max": l_max,
                "c_lmax": float(c[-1]), "c_min": float(np.min(c)),
                "iact_upper_bound": bool(any(ess_flags.values())), "flags": ess_flags,
                "between_chain_ess": ess_between, "between_chain_ess_per_s": ess_between / (ms_step / 1e3),
                "iact_over_between": ratio},
        "acceptance_note": "adaptation per Algorithm 2 (M_A=500) from the pilot beta",
        "mean_error_to_truth_frobenius": float(np.sqrt(np.sum(np.abs(pool["mean"] - prob.truth.density_matrix())
                                                               ** 2))),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "kernel": f"k_chains<Q={Q}>", "kernel_ms": ms_kernel,
                     "flop_per_chain_step": flop, "chain_steps_per_launch": chain_steps,
                     "all_arith_flop_per_chain_step": flop_all,
                     "all_arith_frac": flop_all * chain_steps / (ms_kernel / 1e3) / 1e12 / PEAK_FP64_TFLOPS,
                     "valu_issue": valu_issue(khash, f"chain_kernel_q{Q}_{args.config}",
                                              chain_steps / (ms_kernel / 1e3)),
                     "kernel_source_hash": khash},
    }
    if not args.no_forms:
        print("[bench] chosen forms", file=sys.stderr, flush=True)
        out["forms"] = chosen_forms(qst, torch, np, prob, cfg, record, pool, ms_step, tau, ess_between)
        if Q <= 4:
            print("[bench] Algorithm 1 (Bures draw)", file=sys.stderr, flush=True)
            out["forms"]["bures"] = bures_form(qst, torch, np, prob, cfg, pool)
            print("[bench] Dirichlet weights and user POVMs", file=sys.stderr, flush=True)
            out["forms"].update(option_rates(qst, synth, torch, prob, cfg))
        print("[bench] uneven batch", file=sys.stderr, flush=True)
        out["forms"]["uneven_batch"] = uneven_batch(qst, synth, torch, np)
        if not args.no_delayed:
            from paper_2501_17334_amd import surrogate
            print("[bench] delayed acceptance (5-qubit workload)", file=sys.stderr, flush=True)
            out["forms"]["delayed_acceptance"] = delayed_acceptance(qst, surrogate, synth, torch, np)
    if args.config == "c3" and not args.no_dense_gemm:
        out["dense_gemm"] = dense_gemm_rates(qst, synth, torch, prob)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds, ess_per_chain_step=n_eff / chain_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
