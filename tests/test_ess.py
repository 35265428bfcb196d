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
