"""The scaling study's plumbing on a small case: per-chain moment sums pool
to the library's own Eq. (BME2) estimate, the reference entry has zero
error, and every reported quantity is in range."""
import numpy as np
import pytest
import torch

from paper_2501_17334_amd import qst, study, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_chain_moments_pool_to_the_library_estimate():
    prob = synth.make_problem("w_2")
    P = qst.Problem(2, prob.counts)
    r = study.run_thinning(P, dict(seed=3, beta0=0.1, adapt_every=50), 4, 128, 96, 16, torch)
    assert np.all(r["n_stored"] == 128)
    est = study.unpack(r["s1"].sum(0) / r["n_stored"].sum())
    assert np.abs(est - P.pool()["mean"]).max() < 1e-14
    assert r["tau"] > 0.0
    P.close()


def test_small_study():
    prob = synth.make_problem("w_1")
    out = study.study(1, prob.counts, prob.truth.density_matrix(), T_list=[1, 4], N=64, R_max=64,
                      record_chains=16, seed=prob.seed)
    assert out["R"] == [1, 2, 4, 8, 16, 32, 64]
    last = out["runs"][-1]
    assert last["eps_f2"][-1] == 0.0 and abs(last["infidelity_to_reference"][-1]) < 1e-12
    for run in out["runs"]:
        assert np.all(np.isfinite(run["eps_f2"])) and run["tau"] > 0.0
        assert all(-1e-12 <= v <= 1.0 for v in run["infidelity_to_truth"])
    assert 0.0 < out["reference_fidelity_to_truth"] <= 1.0
