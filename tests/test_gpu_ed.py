"""Monte Carlo averages of the GPU chains against exact diagonalisation at
N_phi = 2 (Fock space of 8 modes): the thermal expectation of m^2_SO(5) of
the Fierz Hamiltonian, Tr[e^{-beta H} m^2] / Tr e^{-beta H}, must agree with
the average over configurations within the statistical error (plus the
Trotter error O(dtau^2), checked by halving dtau)."""
import numpy as np
import pytest

from oracle import fock
from oracle.model import Model, Q_BZ, gamma_matrices, momentum_set

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
