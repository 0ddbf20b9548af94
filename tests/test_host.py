"""CPU tests of the host side: the C ABI library loads and exports every
declared symbol, parameter validation needs no GPU, and the autocorrelation
analysis matches closed forms."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2605_03700_amd", "libcfqmc.so")
HEADER = os.path.join(ROOT, "include", "cfqmc.h")


def declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(cfqmc_[A-Za-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("library not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_header():
    from paper_2605_03700_amd import cfqmc
    assert set(cfqmc.EXPORTS) == set(declared_functions())


def test_param_struct_layout_and_validation(lib):
    from paper_2605_03700_amd import cfqmc
    L = cfqmc.load()
    p = cfqmc.Params()
    L.cfqmc_default_params(ctypes.byref(p))
    assert p.n_phi == 6 and abs(p.r0 - 0.574) < 1e-15 and abs(p.deps - 0.1) < 1e-15
    assert p.exp_squarings == 2 and p.tile_cfg == -1 and p.n_chains == 1 and p.sweep_graph == 1
    h = ctypes.c_void_p()
    for field, bad in [("n_phi", 0), ("n_phi", 141), ("l_tau", 0), ("dtau", -1.0), ("eps0", 0.0),
                       ("n_chains", 0), ("precision", 7), ("tile_cfg", 20), ("n_stab", 0),
                       ("sweep_graph", 2), ("sweep_graph", -1)]:
        q = cfqmc.Params()
        L.cfqmc_default_params(ctypes.byref(q))
        setattr(q, field, bad)
        assert L.cfqmc_create(ctypes.byref(q), None, ctypes.byref(h)) == -1, field
    q = cfqmc.Params()
    L.cfqmc_default_params(ctypes.byref(q))
    q.q_mode = 3       # explicit list missing
    assert L.cfqmc_create(ctypes.byref(q), None, ctypes.byref(h)) == -1
    assert L.cfqmc_destroy(None) == -1
    # the dense 4N form and the exact drift are declared and not implemented
    assert p.dense4n == 0 and p.exact_drift == 0
    for field, val, rc in [("dense4n", 1, -6), ("exact_drift", 1, -6), ("dense4n", 2, -1), ("exact_drift", -1, -1)]:
        q = cfqmc.Params()
        L.cfqmc_default_params(ctypes.byref(q))
        setattr(q, field, val)
        h = ctypes.c_void_p()
        assert L.cfqmc_create(ctypes.byref(q), None, ctypes.byref(h)) == rc, field
        assert h.value is None
    # argument checks that need no GPU
    assert L.cfqmc_batch_get(None, 0, ctypes.byref(h), None) == -1
    assert L.cfqmc_batch_sweep_replay(None, 1, None, None) == -1
    assert L.cfqmc_measure_tau_noalloc(None, None, None) == -1
    assert L.cfqmc_launch_config(None, None) == -1
    out = np.empty(2)
    assert L.cfqmc_green_maxdiff(None, None, 4, 1, None, out.ctypes.data_as(ctypes.c_void_p)) == -1
    assert L.cfqmc_slmc_grad_check(None, None, 1, None, None) == -1


def test_tau_int_ar1_closed_form():
    """AR(1) x_t = r x_{t-1} + e_t has tau_int = (1+r)/(2(1-r))."""
    from paper_2605_03700_amd.analysis import tau_int
    rng = np.random.default_rng(0)
    r = 0.8
    n = 200000
    e = rng.standard_normal(n)
    x = np.empty(n)
    x[0] = e[0]
    for t in range(1, n):
        x[t] = r * x[t - 1] + e[t]
    t, _ = tau_int(x)
    assert abs(t - (1 + r) / (2 * (1 - r))) < 0.3
    w, _ = tau_int(rng.standard_normal(50000))
    assert abs(w - 0.5) < 0.05


def test_product_path_has_no_oracle_import():
    """The package never imports the oracle (test infrastructure only)."""
    pkg = os.path.join(ROOT, "paper_2605_03700_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "oracle" not in re.findall(r"^\s*(?:from|import)\s+(\w+)", src, re.M), fn


def test_tau_int_pooled_ar1_many_short_chains():
    """Pooled over 400 independent AR(1) chains of 40 steps the estimator
    recovers (1+r)/(2(1-r)); white noise gives 1/2."""
    from paper_2605_03700_amd.analysis import tau_int_pooled
    rng = np.random.default_rng(3)
    r = 0.5
    chains = []
    for _ in range(400):
        x = np.empty(40)
        x[0] = rng.standard_normal() / np.sqrt(1 - r * r)
        for t in range(1, 40):
            x[t] = r * x[t - 1] + rng.standard_normal()
        chains.append(x)
    tau, _, closed = tau_int_pooled(chains)
    assert closed and abs(tau - 1.5) < 0.25
    w, _, closed = tau_int_pooled([rng.standard_normal(40) for _ in range(400)])
    assert closed and abs(w - 0.5) < 0.1


def test_tau_int_pooled_removes_a_shared_drift_and_flags_short_series():
    """A relaxation common to all chains (x_t = a e^{-t/5} + AR(1) noise, the
    same a for every chain) does not enter tau_int; a series much shorter
    than its autocorrelation time reports an open window (a lower bound)."""
    from paper_2605_03700_amd.analysis import tau_int_pooled
    rng = np.random.default_rng(4)
    r, n = 0.5, 40
    drift = 10.0 * np.exp(-np.arange(n) / 5.0)
    chains = []
    for _ in range(400):
        x = np.empty(n)
        x[0] = rng.standard_normal() / np.sqrt(1 - r * r)
        for t in range(1, n):
            x[t] = r * x[t - 1] + rng.standard_normal()
        chains.append(x + drift)
    tau, _, closed = tau_int_pooled(chains)
    assert closed and abs(tau - 1.5) < 0.25
    # r = 0.98: tau_int = 49.5 steps, far beyond 20-step series
    slow = []
    for _ in range(200):
        x = np.empty(20)
        x[0] = rng.standard_normal() / np.sqrt(1 - 0.98 ** 2)
        for t in range(1, 20):
            x[t] = 0.98 * x[t - 1] + rng.standard_normal()
        slow.append(x)
    tau, w, closed = tau_int_pooled(slow)
    assert not closed and w == 19 and tau < 49.5


def test_gap_fit_recovers_a_cosh_correlator():
    """A cosh(Delta (tau - beta/2)) (+ constant) on the periodic interval: the
    effective gap is Delta at every tau and the fit returns Delta; pure
    power-law gaps Delta = c N^{-z/2} give z back."""
    from paper_2605_03700_amd.analysis import dynamic_exponent, effective_gap, fit_gap
    L, dtau, d, a = 120, 0.1, 0.8, 0.3
    tau = np.arange(L + 1) * dtau
    c = a * np.cosh(d * (tau - 0.5 * L * dtau))
    assert np.allclose(effective_gap(c, dtau), d, rtol=1e-9)
    got = fit_gap(c, dtau, 10)
    assert abs(got[0] - d) < 1e-8 and abs(got[1] - a) < 1e-8
    got = fit_gap(c + 0.05, dtau, 5, constant=True)
    assert abs(got[0] - d) < 1e-6 and abs(got[2] - 0.05) < 1e-6
    rng = np.random.default_rng(1)
    noisy = c * (1.0 + 1e-3 * rng.standard_normal(c.size))
    assert abs(fit_gap(noisy, dtau, 10)[0] - d) < 0.02
    n = np.array([16, 36, 64, 100, 144])
    z, _ = dynamic_exponent(n, 2.0 * n ** -0.5)
    assert abs(z - 1.0) < 1e-12


def test_order_parameters_and_correlation_ratio():
    """Component sums and normalisations on hand-made S^i: all components
    equal gives m^2_SO(5) = m^2_VBS = m^2_AFM; a flat S(q) gives R = 0 and a
    delta peak at Q gives R = 1."""
    from paper_2605_03700_amd.analysis import correlation_ratio, order_parameters
    n = 6
    s = np.full(5, 7.2) + 0.3j
    a, b, c = order_parameters(s, n)
    assert abs(a - 7.2 / 36) < 1e-15 and abs(b - a) < 1e-15 and abs(c - a) < 1e-15
    s2 = np.array([[2.0, 4.0, 1.0, 1.0, 4.0]])
    a, b, c = order_parameters(s2, 2)
    assert np.allclose([a[0], b[0], c[0]], [12.0 / 20, 6.0 / 8, 6.0 / 12])
    assert correlation_ratio(3.0, 3.0) == 0.0 and correlation_ratio(3.0, 0.0) == 1.0
    assert abs(correlation_ratio(4.0, 1.0) - 0.75) < 1e-15


@pytest.mark.parametrize("n_phi", [1, 2, 5, 12, 33])
def test_sphere_weight_table_matches_the_oracle(n_phi):
    """The library's sphere weight table (three-term recursion of the 3j
    symbols in extended precision, host code) against the oracle's exact
    Racah evaluation of the printed density operator."""
    from oracle.sphere import density_matrix
    from paper_2605_03700_amd.cfqmc import sphere_weights
    W = sphere_weights(n_phi)
    for l in range(n_phi):
        for m in range(n_phi):
            D = density_matrix(l, m, n_phi) if m <= l else np.zeros((n_phi, n_phi))
            ref = np.array([D[r, r + m].real if r + m < n_phi else 0.0 for r in range(n_phi)])
            assert np.abs(W[l, m] - ref).max() < 1e-14, (l, m)


def test_host_only_entry_points_reject_bad_arguments():
    """Host-only calls of the C ABI validate their arguments (no device use)."""
    import ctypes
    from paper_2605_03700_amd.cfqmc import load
    lib = load()
    buf = np.zeros(8)
    assert lib.cfqmc_sphere_weights(0, buf.ctypes.data) == -1          # CFQMC_EINVAL
    assert lib.cfqmc_sphere_weights(289, buf.ctypes.data) == -1
    assert lib.cfqmc_sphere_weights(2, None) == -1
    assert lib.cfqmc_sphere_weights(2, buf.ctypes.data) == 0
    assert abs(abs(buf[0]) - 0.5) < 1e-15                                # n_{0,0} = +-1/2 on the orbitals


def test_product_path_fails_loudly_without_the_library(monkeypatch, tmp_path):
    """Without the built HIP library the binding raises at load and at context
    creation: there is no CPU fallback."""
    from paper_2605_03700_amd import cfqmc
    monkeypatch.setattr(cfqmc, "_lib", None)
    monkeypatch.setattr(cfqmc, "LIB_PATH", str(tmp_path / "missing" / "libcfqmc.so"))
    with pytest.raises(RuntimeError, match="not found"):
        cfqmc.load()
    with pytest.raises(RuntimeError, match="not found"):
        cfqmc.CFQMC(n_phi=4, l_tau=8)


def _fss_data(u_c, d_s, d_v, noise, seed):
    """Synthetic correlation ratios and order parameters obeying the scaling forms
    exactly (cubic scaling function), at the paper's torus sizes and u range."""
    sizes = [16, 20, 24, 28, 32, 40, 48, 56, 64, 72, 96, 112, 128, 140]
    us = np.linspace(0.17, 0.23, 9)
    U, N = np.meshgrid(us, sizes, indexing="ij")
    U, N = U.ravel(), N.ravel().astype(float)
    x = (U / u_c - 1.0) * np.sqrt(N) ** (3.0 - d_s)
    rng = np.random.default_rng(seed)
    R = 0.5 - 0.8 * x + 0.3 * x ** 2 + 0.4 * x ** 3 + noise * rng.standard_normal(x.size)
    m2 = (0.9 - 0.5 * x + 0.2 * x ** 2 - 0.1 * x ** 3) * N ** (-d_v) * (1 + noise * rng.standard_normal(x.size))
    return U, N, R, m2


def test_fss_grid_scan_recovers_known_critical_point():
    """Results eqs. finite-size-scaling-R/-m: on data generated with (u_c, Delta_s)
    = (0.195, 2.65) and a cubic scaling function the R^2-optimised scan over a
    grid containing the truth returns it with R^2 = 1 (exact data), also for the
    order parameter at fixed Delta_v; with 1% noise it stays within one grid step;
    a wrong Delta_s or u_c lowers R^2."""
    from paper_2605_03700_amd.analysis import data_collapse, fss_collapse_r2, fss_grid_scan
    ucg = np.round(np.arange(0.175, 0.2151, 0.005), 4)
    dsg = np.round(np.arange(2.3, 3.001, 0.05), 4)
    U, N, R, m2 = _fss_data(0.195, 2.65, 0.51, 0.0, 1)
    r2map, (uc, ds, r2) = fss_grid_scan(U, N, R, ucg, dsg)
    assert r2map.shape == (ucg.size, dsg.size)
    assert abs(uc - 0.195) < 1e-9 and abs(ds - 2.65) < 1e-9 and r2 > 1 - 1e-12
    _, (uc, ds, r2) = fss_grid_scan(U, N, m2, ucg, dsg, delta_v=0.51)
    assert abs(uc - 0.195) < 1e-9 and abs(ds - 2.65) < 1e-9 and r2 > 1 - 1e-12
    assert fss_collapse_r2(U, N, R, 0.195, 2.3)[0] < r2 - 1e-3
    assert fss_collapse_r2(U, N, R, 0.21, 2.65)[0] < r2 - 1e-3
    U, N, R, m2 = _fss_data(0.195, 2.65, 0.51, 0.01, 2)
    _, (uc, ds, _) = fss_grid_scan(U, N, R, ucg, dsg)
    assert abs(uc - 0.195) <= 0.005 + 1e-9 and abs(ds - 2.65) <= 0.1 + 1e-9
    x, Y, F, r2c = data_collapse(U, N, R, uc, ds)
    assert x.shape == Y.shape == F.shape and r2c > 0.99


def test_cpu_baseline_times_several_moves():
    """The host oracle's rate takes the slice-move time as the difference of
    two separately timed runs (set-up plus k moves, set-up alone), so k must
    be large enough for the moves to stand above the set-up's run-to-run
    noise: at least four moves, up to every slice of the chain."""
    import bench
    r = bench._cpu_rate(4, 8, 0.1, 1.5, seconds=2.0, sphere=False)
    k = int(re.search(r"first (\d+) slice moves", r["sample"]).group(1))
    assert 4 <= k <= 8
    assert np.isfinite(r["value"]) and r["value"] > 0
    assert r["kind"] == "oracle" and r["unit"] == "field updates/s"
