"""Autocorrelation analysis of Monte Carlo time series (host side).

Integrated autocorrelation time with Sokal's automatic window (Madras & Sokal
1988; Wolff 2004 uses the same windowing idea): tau_int(W) = 1/2 + sum_{t=1}^{W}
rho(t), choosing the smallest W with W >= c * tau_int(W), c = 5.
Independent samples per second = sweeps per second / (2 tau_int).
"""
import numpy as np


def autocorr(x):
    """Normalised autocorrelation rho(t) of a 1-D series (FFT, zero padded)."""
    x = np.asarray(x, dtype=float)
    n = x.size
    if n < 2:
        return np.ones(1)
    y = x - x.mean()
    f = np.fft.rfft(y, 2 * n)
    ac = np.fft.irfft(f * np.conj(f))[:n]
    if ac[0] <= 0:
        return np.ones(1)
    return ac / ac[0]


def tau_int(x, c=5.0):
    """Integrated autocorrelation time (in units of the series step) and the window."""
    rho = autocorr(x)
    n = rho.size
    if n < 2:
        return 0.5, 0
    tau = 0.5
    for w in range(1, n):
        tau += rho[w]
        if w >= c * tau:
            return max(tau, 0.5), w
    return max(tau, 0.5), n - 1


def tau_int_pooled(series, c=5.0):
    """tau_int of many equally long series of one observable from independent
    chains of one ensemble. Deviations are taken from the ensemble mean at each
    step (the mean over chains of that sweep), which removes a drift that all
    chains share, such as the relaxation from a common initial distribution,
    and does not bias short series as per-chain means do; over C chains it
    scales every autocovariance by the same factor 1 - 1/C, so rho is
    unchanged. The autocovariance at lag t is averaged over chains and over
    the n - t pairs of each, normalised and windowed as in tau_int.
    Returns (tau_int, window, closed): closed is False when no window up to
    the series length satisfies W >= c tau_int, and tau_int is then a lower
    bound (the series is too short for the slowest mode it contains)."""
    xs = [np.asarray(x, dtype=float) for x in series if len(x) > 1]
    if not xs:
        return 0.5, 0, False
    n = min(x.size for x in xs)
    X = np.stack([x[:n] for x in xs])
    Y = X - X.mean(axis=0, keepdims=True) if X.shape[0] > 1 else X - X.mean()
    f = np.fft.rfft(Y, 2 * n, axis=1)
    acc = np.fft.irfft(f * np.conj(f), axis=1)[:, :n].sum(axis=0) / (n - np.arange(n))
    if acc[0] <= 0:
        return 0.5, 0, False
    rho = acc / acc[0]
    tau = 0.5
    for w in range(1, n):
        tau += rho[w]
        if w >= c * tau:
            return max(tau, 0.5), w, True
    return max(tau, 0.5), n - 1, False


def independent_samples_per_s(sweeps_per_s, series_list):
    """sweeps/s divided by 2 tau_int, tau_int the maximum over the given series."""
    taus = [tau_int(s)[0] for s in series_list if len(s) > 1]
    t = max(taus) if taus else 0.5
    return sweeps_per_s / (2.0 * t), t
