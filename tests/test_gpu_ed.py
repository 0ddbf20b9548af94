"""Monte Carlo averages of the GPU chains against exact diagonalisation at
N_phi = 2 (Fock space of 8 modes): thermal expectations of the Fierz
Hamiltonian (eq. newmodel), Tr[e^{-beta H} O] / Tr e^{-beta H}, must agree
with the averages over configurations within the statistical error, after
removing the Trotter error O(dtau^2) (Methods, Trotter decomposition): m^2_SO(5)
at beta = 4 for two steps, and <H>, the five S^i_{q=0} and m^2_SO(5) at
beta = 1, 2, 4 extrapolated to dtau -> 0 from dtau = 0.1 and 0.05."""
import numpy as np
import pytest

from oracle import fock
from oracle.model import Model, Q_BZ, gamma_matrices, momentum_set
from oracle.observables import fierz_energy

pytestmark = pytest.mark.gpu


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_03700_amd import CFQMC
    return CFQMC


def _ed_m2(n, u, beta):
    cs = fock.annihilators(4 * n)
    m = Model(n, 2, 0.1, u0=1.0, uk=u, un=u, q_mode=Q_BZ)
    H = fock.hamiltonian_fierz(cs, n, momentum_set(n, Q_BZ), m.g)
    ops = [fock.density_operator(cs, n, 0, 0, gm, False) for gm in gamma_matrices()]
    M2 = sum(o @ o for o in ops) / (5 * n * n)
    return fock.thermal_expectation(H, M2, beta), float(np.trace(M2).real / M2.shape[0])


@pytest.mark.parametrize("dtau", [0.05, 0.025])
def test_m2_matches_exact_diagonalisation(dtau):
    CFQMC = _gpu()
    n, u, beta, nch = 2, 5.0, 4.0, 256
    L = int(round(beta / dtau))
    ed, inf_t = _ed_m2(n, u, beta)
    assert ed > 1.5 * inf_t                       # the interaction moves m^2 well away from infinite temperature
    g = CFQMC(n_phi=n, l_tau=L, dtau=dtau, u0=1.0, uk=u, un=u, q_mode=Q_BZ, n_stab=10, n_chains=nch, seed=77,
              eps0=0.5)
    g.init_fields()
    g.sweep(40)
    n0 = len(g.series(0, "m2"))
    g.sweep(160)
    means = np.array([np.mean(g.series(k, "m2")[n0:]) for k in range(nch)])
    mc, err = means.mean(), means.std(ddof=1) / np.sqrt(nch)
    g.close()
    # Trotter error O(dtau^2): allow 2% at dtau = 0.05, 0.5% at 0.025, on top of 4 sigma
    tol = 4.0 * err + (0.02 if dtau > 0.03 else 0.005) * ed
    print("dtau %g: MC %.6g +- %.2g, ED %.6g, infinite T %.6g" % (dtau, mc, err, ed, inf_t))
    assert abs(mc - ed) < tol, (mc, err, ed)


def _mc(n, u, beta, dtau, nch, therm, meas, seed, qs, g_coupl):
    """Per-chain averages over `meas` sweeps after `therm`: <H> by Wick's theorem
    from the chains' equal-time G every second sweep, S^i_{q=0} (i = 1..5) every
    sweep, m^2_SO(5) from the per-sweep series. Returns {name: (mean, stderr)}
    with errors from the spread of the independent chains."""
    CFQMC = _gpu()
    L = int(round(beta / dtau))
    g = CFQMC(n_phi=n, l_tau=L, dtau=dtau, u0=1.0, uk=u, un=u, q_mode=Q_BZ, n_stab=10, n_chains=nch, seed=seed,
              eps0=0.5, exp_squarings=6)
    g.init_fields()
    g.sweep(therm)
    n0 = len(g.series(0, "m2"))
    e = np.zeros(nch)
    s = np.zeros((nch, 5))
    ne = 0
    for sw in range(meas):
        g.sweep(1)
        s += g.structure_factors([(0, 0)])[:, 0, :].real
        if sw % 2 == 0:
            G = np.array([g.measure_G(k, 0)[:2 * n, :2 * n] for k in range(nch)])
            e += fierz_energy(G, n, qs, g_coupl).real
            ne += 1
    m2 = np.array([np.mean(g.series(k, "m2")[n0:]) for k in range(nch)])
    g.close()
    cols = {"E": e / ne, "m2": m2}
    for i in range(5):
        cols["S%d" % (i + 1)] = s[:, i] / meas
    return {k: (v.mean(), v.std(ddof=1) / np.sqrt(nch)) for k, v in cols.items()}


@pytest.mark.parametrize("beta", [1.0, 2.0, 4.0])
def test_energy_structure_factors_extrapolated_to_zero_dtau(beta):
    n, u = 2, 5.0
    cs = fock.annihilators(4 * n)
    m = Model(n, 2, 0.1, u0=1.0, uk=u, un=u, q_mode=Q_BZ)
    qs = momentum_set(n, Q_BZ)
    H = fock.hamiltonian_fierz(cs, n, qs, m.g)
    ops = [fock.density_operator(cs, n, 0, 0, gm, False) for gm in gamma_matrices()]
    ed = {"E": fock.thermal_expectation(H, H, beta)}
    for i, o in enumerate(ops):
        ed["S%d" % (i + 1)] = fock.thermal_expectation(H, o @ o, beta)
    ed["m2"] = sum(ed["S%d" % (i + 1)] for i in range(5)) / (5 * n * n)
    r1 = _mc(n, u, beta, 0.1, 256, 40, 100, 11, qs, m.g)
    r2 = _mc(n, u, beta, 0.05, 256, 40, 100, 12, qs, m.g)
    for k, v in ed.items():
        # X(dtau) = X_0 + c dtau^2: X_0 = (4 X(dtau/2) - X(dtau)) / 3
        x0 = (4.0 * r2[k][0] - r1[k][0]) / 3.0
        err = np.sqrt(16.0 * r2[k][1] ** 2 + r1[k][1] ** 2) / 3.0
        print("beta %g %s: dtau 0.1 %.6g, 0.05 %.6g, extrapolated %.6g +- %.2g, ED %.6g"
              % (beta, k, r1[k][0], r2[k][0], x0, err, v))
        assert abs(x0 - v) < 4.0 * err + 2e-3 * abs(v), (beta, k, x0, err, v)
    # the interaction splits the channels: S^{1,2} and S^{3,4,5} differ in ED
    assert abs(ed["S1"] - ed["S3"]) > 10 * max(r1["S1"][1], r1["S3"][1])
