"""User POVM elements on the dense MFMA path against the oracle's direct
p_m = Tr(Pi_m rho).

* chains on random-basis measurements (2, 3 and 4 qubits) and on the qubit
  SIC-POVM (four elements, padded to six rows): per-step log L within 1e-10
  relative while the decisions agree, final states equal;
* log L of given states: the Pauli settings given as POVM elements against
  the library's own Pauli matrix within 1e-12 relative (FP64), and the FP32
  form within 1e-6 of the total count;
* what is not built is refused.
"""
import itertools

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2501_17334_amd import qst, synth
from tests.gpu_util import first_near_step

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _chains(prob, R, T, beta0, precision="fp64"):
    Q = prob.n_qubits
    P = qst.Problem(Q, prob.counts, precision=precision, povm=prob.povm)
    tr = dict(chains=R, llprop=torch.full((R, T), float("nan"), dtype=torch.float64, device="cuda"),
              logu=torch.zeros((R, T), dtype=torch.float64, device="cuda"),
              accept=torch.zeros((R, T), dtype=torch.int8, device="cuda"))
    P.run(qst.RunConfig(n_chains=R, n_steps=T, seed=prob.seed, beta0=beta0, adapt_every=0), trace=tr)
    torch.cuda.synchronize()
    ch = O.Chains(Q, prob.counts, O.RunParams(n_chains=R, n_steps=0, seed=prob.seed, beta0=beta0, adapt_every=0,
                                              trace_chains=R, povm=prob.povm))
    ll0 = ch.ll.copy()
    o = ch.run(T)
    return P, ch, o, ll0, tr["llprop"].cpu().numpy(), tr["accept"].cpu().numpy()


@pytest.mark.parametrize("name", ["sic_1", "bases_2", "bases_3", "bases_4"])
def test_povm_chains_match_oracle(name):
    prob = synth.sic_qubit_problem() if name == "sic_1" else synth.random_bases_problem(int(name[-1]))
    Q = prob.n_qubits
    R, T, beta0 = {1: (32, 300, 0.1), 2: (32, 200, 0.05), 3: (16, 100, 0.03), 4: (16, 60, 0.02)}[Q]
    print(f"[povm] {name} R={R} T={T}", flush=True)
    P, ch, o, ll0, g_ll, g_acc = _chains(prob, R, T, beta0)
    stop = first_near_step(o["trace_llprop"], g_ll, o["trace_logu"], ll0, o["trace_accept"])
    worst = 0.0
    for r in range(R):
        s = stop[r]
        rel = np.abs(o["trace_llprop"][r, :s] - g_ll[r, :s]) / np.abs(o["trace_llprop"][r, :s])
        if s:
            worst = max(worst, float(rel.max()))
        assert np.all(rel <= 1e-10), (r, rel.max())
        assert np.array_equal(o["trace_accept"][r, :s], g_acc[r, :s]), r
    x = P.state()[0]
    clean = stop == T
    assert np.allclose(x[clean], ch.x[clean], rtol=1e-9, atol=1e-9)
    print(f"  max relative |dlogL| {worst:.2e}", flush=True)


def _pauli_povm(Q):
    s2 = 1 / np.sqrt(2)
    eig = {0: [np.array([s2, s2]), np.array([s2, -s2])], 1: [np.array([s2, 1j * s2]), np.array([s2, -1j * s2])],
           2: [np.array([1.0, 0.0]), np.array([0.0, 1.0])]}
    out = []
    for s in itertools.product(range(3), repeat=Q):
        for b in itertools.product(range(2), repeat=Q):
            v = np.array([1.0 + 0j])
            for q in range(Q):
                v = np.kron(v, eig[s[q]][b[q]])
            out.append(np.outer(v, v.conj()))
    return np.stack(out)


@pytest.mark.parametrize("Q", [2, 4])
def test_pauli_settings_given_as_povm(Q):
    prob = {2: synth.make_problem("c2"), 4: synth.make_problem("c3")}[Q]
    D = 2 ** Q
    rng = np.random.default_rng(60 + Q)
    rhos = np.stack([synth.random_density_matrix(D, rng, rank=int(rng.integers(1, D + 1))) for _ in range(40)])
    dev = torch.from_numpy(np.ascontiguousarray(np.stack([rhos.real, rhos.imag], -1))).cuda()
    A = qst.Problem(Q, prob.counts.reshape(-1), povm=_pauli_povm(Q))
    B = qst.Problem(Q, prob.counts, path="dense")
    out_a = torch.zeros(40, dtype=torch.float64, device="cuda")
    out_b = torch.zeros(40, dtype=torch.float64, device="cuda")
    A.loglik(dev, out_a)
    B.loglik(dev, out_b)
    a, b = out_a.cpu().numpy(), out_b.cpu().numpy()
    assert np.all(np.abs(a - b) <= 1e-12 * np.abs(b))
    out_f = torch.zeros(40, dtype=torch.float64, device="cuda")
    A.loglik(dev, out_f, precision="fp32")
    assert np.all(np.abs(out_f.cpu().numpy() - b) <= 1e-6 * prob.counts.sum())


def test_povm_refusals():
    prob = synth.random_bases_problem(2)
    for kw in (dict(path="kron"), dict(precision="bf16x3"), dict(param="bures")):
        with pytest.raises(qst.QstError):
            qst.Problem(2, prob.counts, povm=prob.povm, **kw)
    bad = prob.povm.copy()
    bad[0, 0, 1] += 0.5            # no longer Hermitian
    with pytest.raises(qst.QstError) as e:
        qst.Problem(2, prob.counts, povm=bad)
    assert e.value.status == qst.QST_ERR_INVALID
    P = qst.Problem(2, prob.counts, povm=prob.povm)
    rho = torch.zeros((1, 4, 4, 2), dtype=torch.float64, device="cuda")
    rho[0, :, :, 0] = torch.eye(4, dtype=torch.float64) / 4
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(qst.QstError):
        P.loglik(rho, out, path="kron")
