"""ESS estimator checks against closed forms (CPU)."""
import numpy as np
import pytest

from paper_1210_5128_amd import ess


def ar1(rho, n, seed):
    rng = np.random.default_rng(seed)
    e = rng.standard_normal(n)
    x = np.empty(n)
    x[0] = e[0] / np.sqrt(1 - rho * rho)
    for t in range(1, n):
        x[t] = rho * x[t - 1] + e[t]
    return x


@pytest.mark.parametrize("rho", [0.0, 0.5, 0.9])
def test_ar1_ess_matches_closed_form(rho):
    # AR(1): integrated autocorrelation time (1 + rho) / (1 - rho)
    n = 200000
    got = ess.ess_chain(ar1(rho, n, seed=int(rho * 10)))
    want = n * (1 - rho) / (1 + rho)
    assert got == pytest.approx(want, rel=0.08)


def test_ess_sums_over_chains_and_handles_constants():
    x = np.stack([ar1(0.5, 20000, s) for s in range(4)])
    per = [ess.ess_chain(r[4000:]) for r in x]
    assert ess.ess(x) == pytest.approx(sum(per))
    assert ess.ess_chain(np.ones(100)) == 1.0


def test_split_rhat():
    x = np.stack([ar1(0.3, 5000, s) for s in range(4)])
    assert ess.split_rhat(x) < 1.02
    y = x.copy()
    y[0] += 5.0
    assert ess.split_rhat(y) > 1.5


def test_multichain_ess_matches_closed_form_when_chains_agree():
    # four AR(1) chains of the same process: the pooled ESS is the sum
    n, rho = 50000, 0.5
    x = np.stack([ar1(rho, n, 10 + s) for s in range(4)])
    want = 4 * n * (1 - rho) / (1 + rho)
    assert ess.ess_multichain(x) == pytest.approx(want, rel=0.08)
    # rank normalisation is monotone, so the bulk ESS of a Gaussian process stays close
    assert ess.ess_bulk(x, burn=0.0) == pytest.approx(want, rel=0.1)
    assert ess.rhat_rank(x) < 1.01


def test_multichain_ess_collapses_when_chains_disagree():
    # chains stuck at different levels: the summed per-chain ESS does not see it,
    # the pooled estimate and R-hat do
    x = np.stack([ar1(0.5, 20000, 20 + s) + 3.0 * s for s in range(4)])
    assert ess.ess(x) > 20000
    assert ess.ess_multichain(x) < 100
    assert ess.rhat_rank(x) > 1.5
    # a drifting chain: its two halves disagree
    drift = ar1(0.5, 20000, 30) + np.linspace(0, 20, 20000)
    assert ess.rhat_rank(drift[None, :], burn=0.0) > 1.5


def test_rank_normalize_and_mcse():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((4, 1000))
    z = ess.rank_normalize(x)
    assert z.shape == x.shape
    assert abs(z.mean()) < 1e-12 and z.std() == pytest.approx(1.0, rel=0.01)
    # iid draws: MCSE of the mean = sd / sqrt(S)
    assert ess.mcse_mean(x, burn=0.0) == pytest.approx(x.std() / np.sqrt(x.size), rel=0.1)
    # binary indicators with ties still rank
    b = (rng.random((4, 1000)) < 0.3).astype(float)
    assert np.isfinite(ess.ess_bulk(b)) and ess.rhat_rank(b) < 1.05


def test_agreement_within_mcse():
    a = np.stack([ar1(0.5, 20000, 40 + s) for s in range(4)])
    b = np.stack([ar1(0.5, 20000, 50 + s) for s in range(4)])
    assert ess.agree_within_mcse(a, b)[2]
    assert not ess.agree_within_mcse(a, b + 0.5)[2]
