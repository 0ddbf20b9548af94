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


def effective_gap(c, dtau):
    """Per-tau gap estimate of a bosonic correlator that is periodic in
    imaginary time, C(tau) = A cosh(Delta (tau - beta/2)) at long times:
    C(t-1) + C(t+1) = 2 cosh(Delta dtau) C(t), so
    Delta_eff(t) = arccosh((C(t-1) + C(t+1)) / (2 C(t))) / dtau for
    t = 1..len(c)-2 (NaN where the ratio is below one). c: C at tau = t dtau,
    t = 0..L (C(L) = C(0))."""
    c = np.asarray(c, dtype=float)
    r = (c[:-2] + c[2:]) / (2.0 * c[1:-1])
    out = np.full(r.size, np.nan)
    ok = r >= 1.0
    out[ok] = np.arccosh(r[ok]) / dtau
    return out


def fit_gap(c, dtau, t_lo, t_hi=None, constant=False):
    """Gap Delta_SO5 from the long-time tail of m^2_SO(5)(tau, q=0)
    (Supplementary Note 2: exponential decay at long imaginary times; on the
    periodic interval the decay from both ends adds to A cosh(Delta (tau -
    beta/2))). Least squares of A cosh(Delta (tau - beta/2)) (+ B with
    constant=True) over t_lo <= t <= t_hi (default L - t_lo). Returns
    (Delta, A[, B])."""
    from scipy.optimize import curve_fit
    c = np.asarray(c, dtype=float)
    L = c.size - 1
    t_hi = L - t_lo if t_hi is None else t_hi
    t = np.arange(t_lo, t_hi + 1)
    half = 0.5 * L * dtau
    x = t * dtau - half
    y = c[t]
    d0 = effective_gap(c, dtau)
    d0 = d0[max(t_lo - 1, 0):max(t_lo - 1, 0) + 3]
    d0 = float(np.nanmean(d0)) if np.isfinite(d0).any() else 1.0 / max(half, 1e-9)
    a0 = float(c[L // 2])
    if constant:
        f = lambda x, d, a, b: a * np.cosh(d * x) + b
        p, _ = curve_fit(f, x, y, p0=[d0, a0, 0.0], maxfev=20000)
        return float(abs(p[0])), float(p[1]), float(p[2])
    f = lambda x, d, a: a * np.cosh(d * x)
    p, _ = curve_fit(f, x, y, p0=[d0, a0], maxfev=20000)
    return float(abs(p[0])), float(p[1])


def dynamic_exponent(n_phis, gaps):
    """z from Delta_SO5 ~ (sqrt N_phi)^-z (Supplementary Note 2): slope of the
    least-squares line of ln Delta against ln(1/sqrt N_phi). Returns (z, C)."""
    x = np.log(1.0 / np.sqrt(np.asarray(n_phis, dtype=float)))
    y = np.log(np.asarray(gaps, dtype=float))
    z, c0 = np.polyfit(x, y, 1)
    return float(z), float(c0)


# ------------------------------------------------------------------ order parameters

TORUS_DQ = ((1, 0), (0, 1), (-1, 0), (0, -1))   # smallest non-zero torus momenta (grid units)


def order_parameters(s_q0, n_phi):
    """From S^i_{q=0}, i = 1..5 (last axis): m^2_SO(5) = sum_i S^i / (5 N^2)
    (Results), and, off the SO(5) line, the VBS (i = 1, 2) and AFM
    (i = 3, 4, 5) order parameters normalised the same way,
    m^2_VBS = (S^1 + S^2) / (2 N^2), m^2_AFM = (S^3 + S^4 + S^5) / (3 N^2).
    Returns (m2_so5, m2_vbs, m2_afm)."""
    s = np.real(np.asarray(s_q0))
    n2 = float(n_phi) ** 2
    return (s[..., :5].sum(-1) / (5 * n2), s[..., :2].sum(-1) / (2 * n2), s[..., 2:5].sum(-1) / (3 * n2))


def correlation_ratio(s_Q, s_Q_dq):
    """R = 1 - S(Q + dq) / S(Q) (Results), dq the smallest non-zero momentum;
    arguments are Monte Carlo averages (S(Q + dq) may be averaged over the
    symmetry-equivalent dq first). R -> 1 with long-range order, -> 0 without."""
    return 1.0 - np.real(np.asarray(s_Q_dq)) / np.real(np.asarray(s_Q))


def fss_scaling_variable(u, n_phi, u_c, delta_s):
    """Finite-size scaling variable of the SO(5) line (Results, eqs.
    finite-size-scaling-R and finite-size-scaling-m): x = (u / u_c - 1)
    sqrt(N_phi)^(3 - Delta_s), with sqrt(N_phi) the linear size."""
    u = np.asarray(u, dtype=float)
    n = np.asarray(n_phi, dtype=float)
    return (u / u_c - 1.0) * np.sqrt(n) ** (3.0 - delta_s)


def fss_collapse_r2(u, n_phi, y, u_c, delta_s, delta_v=None, degree=3):
    """Quality of the data collapse at (u_c, Delta_s): the scaled observable
    Y = y (correlation ratio R) or Y = y N_phi^Delta_v (m^2_SO(5), with
    Delta_v given) is fitted by one polynomial F(x) of the given degree (third
    order, as the paper approximates the universal scaling function near u_c)
    in the scaling variable x; returns (R^2 = 1 - SS_res / SS_tot, polynomial
    coefficients, highest power first)."""
    y = np.asarray(y, dtype=float)
    Y = y if delta_v is None else y * np.asarray(n_phi, dtype=float) ** delta_v
    x = fss_scaling_variable(u, n_phi, u_c, delta_s)
    coef = np.polyfit(x, Y, degree)
    res = Y - np.polyval(coef, x)
    tot = Y - Y.mean()
    ss_tot = float(np.dot(tot, tot))
    r2 = 1.0 - float(np.dot(res, res)) / ss_tot if ss_tot > 0 else 0.0
    return r2, coef


def fss_grid_scan(u, n_phi, y, u_c_grid, delta_s_grid, delta_v=None, degree=3):
    """R^2-optimised grid scan over (u_c, Delta_s) (Results, phase structure
    along the SO(5)-symmetric line; Supplementary Note 3): the R^2 map
    [len(u_c_grid)][len(delta_s_grid)] of fss_collapse_r2 and the best
    (u_c, Delta_s, R^2)."""
    r2 = np.empty((len(u_c_grid), len(delta_s_grid)))
    for i, uc in enumerate(u_c_grid):
        for j, ds in enumerate(delta_s_grid):
            r2[i, j] = fss_collapse_r2(u, n_phi, y, uc, ds, delta_v, degree)[0]
    i, j = np.unravel_index(np.argmax(r2), r2.shape)
    return r2, (float(u_c_grid[i]), float(delta_s_grid[j]), float(r2[i, j]))


def data_collapse(u, n_phi, y, u_c, delta_s, delta_v=None, degree=3):
    """Collapsed data at (u_c, Delta_s): (x, Y, fitted F(x), R^2) with x the
    scaling variable and Y the scaled observable of fss_collapse_r2."""
    r2, coef = fss_collapse_r2(u, n_phi, y, u_c, delta_s, delta_v, degree)
    y = np.asarray(y, dtype=float)
    Y = y if delta_v is None else y * np.asarray(n_phi, dtype=float) ** delta_v
    x = fss_scaling_variable(u, n_phi, u_c, delta_s)
    return x, Y, np.polyval(coef, x), r2
