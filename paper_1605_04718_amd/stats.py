"""MCMC output analysis on the host: rank-normalised split-R-hat and bulk /
tail effective sample size (Vehtari, Gelman, Simpson, Carpenter, Buerkner,
"Rank-normalization, folding, and localization: an improved R-hat for
assessing convergence of MCMC", Bayesian Analysis 16(2), 2021), with Geyer's
initial monotone sequence for the autocorrelation sum, and Monte Carlo
standard errors.  These summarise sampler output; they are not a step of
the sampler.
"""
from __future__ import annotations

import numpy as np
from scipy import special


def _split(x: np.ndarray) -> np.ndarray:
    """[chains, draws] -> [2 chains, draws // 2] (first and second halves)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[1] // 2
    return np.concatenate([x[:, :n], x[:, x.shape[1] - n:]], axis=0)


def _rank_normalise(x: np.ndarray) -> np.ndarray:
    flat = x.ravel()
    r = np.empty(flat.size)
    order = np.argsort(flat, kind="mergesort")
    r[order] = np.arange(1, flat.size + 1)
    # average ranks of ties
    vals, inv, cnt = np.unique(flat, return_inverse=True, return_counts=True)
    if np.any(cnt > 1):
        sums = np.bincount(inv, weights=r)
        r = (sums / cnt)[inv]
    z = np.sqrt(2.0) * special.erfinv(2.0 * (r - 0.375) / (flat.size + 0.25) - 1.0)
    return z.reshape(x.shape)


def _autocov(x: np.ndarray) -> np.ndarray:
    """Biased autocovariance of each row, via FFT."""
    m, n = x.shape
    xc = x - x.mean(axis=1, keepdims=True)
    nfft = 1 << (2 * n - 1).bit_length()
    f = np.fft.rfft(xc, nfft, axis=1)
    ac = np.fft.irfft(f * np.conj(f), nfft, axis=1)[:, :n]
    return ac / n


def ess_raw(x: np.ndarray) -> float:
    """Multi-chain ESS of draws x [chains, draws] (no splitting/ranking)."""
    x = np.asarray(x, dtype=np.float64)
    m, n = x.shape
    if n < 4:
        return float("nan")
    acov = _autocov(x)
    mean_var = acov[:, 0].mean() * n / (n - 1)
    var_plus = mean_var * (n - 1) / n
    if m > 1:
        var_plus += x.mean(axis=1).var(ddof=1)
    if not var_plus > 0:
        return float("nan")
    rho = 1.0 - (mean_var - acov.mean(axis=0)) / var_plus
    rho[0] = 1.0
    # Geyer: sum of consecutive pairs while positive, made monotone
    t = 0
    pairs = []
    while t + 1 < n:
        p = rho[t] + rho[t + 1]
        if p <= 0:
            break
        pairs.append(p)
        t += 2
    pairs = np.minimum.accumulate(np.array(pairs)) if pairs else np.array([1.0])
    tau = -1.0 + 2.0 * pairs.sum()
    tau = max(tau, 1.0 / np.log10(m * n + 10))
    return float(m * n / tau)


def ess_bulk(x: np.ndarray) -> float:
    return ess_raw(_rank_normalise(_split(x)))


def ess_tail(x: np.ndarray, prob=(0.05, 0.95)) -> float:
    s = _split(x)
    out = []
    for p in prob:
        q = np.quantile(s, p)
        out.append(ess_raw((s <= q).astype(np.float64)))
    return float(min(out))


def rhat(x: np.ndarray) -> float:
    """Rank-normalised split-R-hat (max of bulk and folded)."""
    s = _split(x)

    def _r(y):
        m, n = y.shape
        w = y.var(axis=1, ddof=1).mean()
        b = n * y.mean(axis=1).var(ddof=1)
        return float(np.sqrt(((n - 1) / n * w + b / n) / w)) if w > 0 else float("nan")

    z = _rank_normalise(s)
    zf = _rank_normalise(np.abs(s - np.median(s)))
    return max(_r(z), _r(zf))


def mcse_mean(x: np.ndarray) -> float:
    x = np.asarray(x, dtype=np.float64)
    return float(x.std(ddof=1) / np.sqrt(ess_raw(_split(x))))


def mcse_quantile(x: np.ndarray, p: float) -> float:
    """MCSE of the p-quantile by the indicator-ESS interval method."""
    x = np.asarray(x, dtype=np.float64)
    s = _split(x)
    ess = ess_raw((s <= np.quantile(s, p)).astype(np.float64))
    if not np.isfinite(ess) or ess <= 0:
        return float("nan")
    from scipy import stats as st
    a = st.beta.ppf(0.1586553, ess * p + 1, ess * (1 - p) + 1)
    b = st.beta.ppf(0.8413447, ess * p + 1, ess * (1 - p) + 1)
    srt = np.sort(x.ravel())
    n = srt.size
    lo = srt[int(np.clip(np.floor(a * n), 0, n - 1))]
    hi = srt[int(np.clip(np.ceil(b * n), 0, n - 1))]
    return float((hi - lo) / 2)


def summary(trace: np.ndarray, names=("a", "b", "ln_gamma", "ln_d")) -> dict:
    """trace [draws, chains, params] -> per-parameter mean, quantiles, ESS, R-hat, MCSE.
    ESS, R-hat and MCSE are NaN for traces of fewer than 8 draws."""
    out = {}
    nan = float("nan")
    for i, nm in enumerate(names[: trace.shape[2]]):
        x = trace[:, :, i].T
        if x.shape[1] < 8:
            out[nm] = dict(mean=float(x.mean()), q025=float(np.quantile(x, 0.025)),
                           q975=float(np.quantile(x, 0.975)), ess_bulk=nan, ess_tail=nan,
                           rhat=nan, mcse_mean=nan)
            continue
        out[nm] = dict(mean=float(x.mean()), q025=float(np.quantile(x, 0.025)),
                       q975=float(np.quantile(x, 0.975)), ess_bulk=ess_bulk(x),
                       ess_tail=ess_tail(x), rhat=rhat(x), mcse_mean=mcse_mean(x))
    return out
