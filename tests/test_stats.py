"""ESS / R-hat against processes with known answers (host code, no GPU)."""
import numpy as np

from paper_1605_04718_amd import stats


def ar1(m, n, rho, seed):
    rng = np.random.default_rng(seed)
    x = np.empty((m, n))
    x[:, 0] = rng.standard_normal(m) / np.sqrt(1 - rho ** 2)
    e = rng.standard_normal((m, n))
    for t in range(1, n):
        x[:, t] = rho * x[:, t - 1] + e[:, t]
    return x


def test_ess_of_iid_draws_is_the_draw_count():
    x = np.random.default_rng(0).standard_normal((8, 2000))
    assert 0.85 * x.size < stats.ess_bulk(x) < 1.15 * x.size


def test_ess_of_ar1_matches_closed_form():
    # integrated autocorrelation time of AR(1): (1 + rho) / (1 - rho)
    for rho in (0.5, 0.9):
        x = ar1(8, 4000, rho, seed=int(rho * 10))
        want = x.size * (1 - rho) / (1 + rho)
        assert 0.8 * want < stats.ess_bulk(x) < 1.2 * want


def test_rhat_detects_unmixed_chains():
    rng = np.random.default_rng(1)
    good = rng.standard_normal((4, 1000))
    assert stats.rhat(good) < 1.01
    bad = good + np.arange(4)[:, None]
    assert stats.rhat(bad) > 1.5


def test_mcse_of_mean_and_quantile_scale_with_ess():
    x = np.random.default_rng(2).standard_normal((4, 4000))
    assert abs(stats.mcse_mean(x) - 1 / np.sqrt(x.size)) < 0.2 / np.sqrt(x.size)
    q = stats.mcse_quantile(x, 0.975)
    assert 0.5 * 0.02 < q < 2 * 0.04
