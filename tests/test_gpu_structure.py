"""GPU parity of the equal-time structure factors S^i_q at non-zero momenta,
on and off the SO(5) line (U_K != U_N), against the FP64 oracle through the C
ABI. Bar: 1e-10 relative."""
import numpy as np
import pytest

import synth
from oracle import dqmc
from oracle.model import Model, Q_BZ, Q_PAPER, gamma_matrices
from oracle.observables import structure_factor

pytestmark = pytest.mark.gpu


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_03700_amd import CFQMC
    return CFQMC


@pytest.mark.parametrize("n_phi,L,nstab,mode", [(4, 8, 4, Q_BZ), (5, 7, 3, Q_PAPER), (6, 40, 10, Q_BZ),
                                                (24, 20, 10, Q_PAPER)])
def test_structure_factors_parity(n_phi, L, nstab, mode):
    CFQMC = _gpu()
    us = [(1.0, 1.0, 1.0), (1.0, 0.5, 1.5), (1.0, 1.5, 0.4)]   # on and off the SO(5) line
    models = [Model(n_phi, L, 0.1, u0=a, uk=b, un=c, q_mode=mode) for (a, b, c) in us]
    phi = np.stack([synth.fields(400 + 3 * k + n_phi, L, models[0].n_q) for k in range(len(us))])
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.1, q_mode=mode, n_stab=nstab, n_chains=len(us), chain_u=us,
              tile_cfg=1)
    g.init_fields(phi)
    qs = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (2, -1), (n_phi - 1, 1), (0, n_phi), (-3, 2)]
    s = g.structure_factors(qs)
    assert s.shape == (len(us), len(qs), 5)
    for k in range(len(us)):
        G = dqmc.green(models[k], phi[k], 0)
        want = np.array([[structure_factor(G, n_phi, gm, qx, qy) for gm in gamma_matrices()] for (qx, qy) in qs])
        err = np.abs(s[k] - want).max() / np.abs(want).max()
        assert err < 1e-10, (k, err)
        s0, _ = g.observables(k)
        assert np.abs(s[k, 0].real - s0).max() < 1e-10 * np.abs(s0).max()
    g.close()


def test_structure_factors_n100_against_the_oracle():
    """N_phi = 100, paper cutoff: S^i_q at the zero, smallest and a large
    momentum within 1e-10 of the oracle."""
    CFQMC = _gpu()
    n_phi, L = 100, 8
    m = Model(n_phi, L, 0.1, u0=1.0, uk=1.5, un=1.5, q_mode=Q_PAPER)
    phi = synth.fields(452, L, m.n_q)
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.1, u0=1.0, uk=1.5, un=1.5, q_mode=Q_PAPER, n_stab=4)
    g.init_fields(phi[None])
    qs = [(0, 0), (1, 0), (0, 1), (7, -5)]
    s = g.structure_factors(qs)
    G = dqmc.green(m, phi, 0)
    want = np.array([[structure_factor(G, n_phi, gm, qx, qy) for gm in gamma_matrices()] for (qx, qy) in qs])
    assert np.abs(s[0] - want).max() / np.abs(want).max() < 1e-10
    g.close()
