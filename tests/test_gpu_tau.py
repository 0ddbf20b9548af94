"""GPU parity of the time-displaced Green's functions and the imaginary-time
SO(5) correlator (Supplementary Note 2) against the FP64 oracle, through the
C ABI. Bar: 1e-10 relative (FP64 in every precision mode)."""
import numpy as np
import pytest

import synth
from oracle import dqmc
from oracle.model import Model, Q_BZ, Q_PAPER
from oracle.observables import so5_correlator

pytestmark = pytest.mark.gpu


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_03700_amd import CFQMC
    return CFQMC


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


CASES = [
    # n_phi, L, n_stab, q_mode, u
    (4, 8, 4, Q_BZ, 1.0),
    (5, 7, 3, Q_PAPER, 1.3),      # odd N, ragged last block (boundaries 0, 3, 6, 7)
    (6, 40, 10, Q_BZ, 1.0),       # the N_phi = 6 workload
]


@pytest.mark.parametrize("n_phi,L,nstab,mode,u", CASES)
def test_displaced_green_parity(n_phi, L, nstab, mode, u):
    CFQMC = _gpu()
    m = Model(n_phi, L, 0.1, u0=1.0, uk=u, un=u, q_mode=mode)
    phi = synth.fields(300 + n_phi, L, m.n_q)
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.1, u0=1.0, uk=u, un=u, q_mode=mode, n_stab=nstab, tile_cfg=1)
    g.init_fields(phi[None])
    Bs = dqmc.propagators(m, phi)
    taus = sorted({t for t in (0, 1, nstab - 1, nstab, nstab + 1, 2 * nstab + 1, L - 1, L) if 0 <= t <= L})
    for tau in taus:
        got = g.green_displaced(0, tau)
        want = dqmc.green_displaced(m, phi, tau, Bs)
        for name, a, b in zip(("G(tau,0)", "G(0,tau)", "G(tau,tau)"), got, want):
            assert rel(a, b) < 1e-10, (name, tau, rel(a, b))
    g.close()


@pytest.mark.parametrize("n_phi,L,nstab,mode,u", CASES)
def test_tau_correlator_parity(n_phi, L, nstab, mode, u):
    """Two chains at different couplings; every tau = 0..L against the oracle's
    Wick evaluation; C(0) equals the equal-time S^i_{q=0} and C(L) = C(0)."""
    CFQMC = _gpu()
    us = [u, 0.5 * u]
    models = [Model(n_phi, L, 0.1, u0=1.0, uk=x, un=x, q_mode=mode) for x in us]
    phi = np.stack([synth.fields(320 + 7 * k + n_phi, L, models[0].n_q) for k in range(2)])
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.1, q_mode=mode, n_stab=nstab, n_chains=2,
              chain_u=[(1.0, x, x) for x in us], tile_cfg=1)
    g.init_fields(phi)
    c, st = g.measure_tau(with_stab=True)
    assert c.shape == (2, L + 1, 5)
    assert st.max() < 1e-10
    for k in range(2):
        Bs = dqmc.propagators(models[k], phi[k])
        G00 = dqmc.green(models[k], phi[k], 0, Bs)
        want = np.array([so5_correlator(*dqmc.green_displaced(models[k], phi[k], t, Bs), G00, n_phi)[0]
                         for t in range(L + 1)])
        assert rel(c[k], want) < 1e-10, rel(c[k], want)
        s, _ = g.observables(k)
        assert np.abs(c[k, 0].real - s).max() < 1e-10 * np.abs(s).max()
        assert rel(c[k, L], c[k, 0]) < 1e-10
    g.close()


def test_tau_correlator_after_mixed_sweeps():
    """In a mixed-precision context after sweeps the pass still runs in FP64:
    against the oracle on the fields the chain holds."""
    CFQMC = _gpu()
    from paper_2605_03700_amd import MIXED
    n_phi, L, nstab, u = 6, 40, 10, 1.0
    m = Model(n_phi, L, 0.1, u0=1.0, uk=u, un=u, q_mode=Q_BZ)
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.1, u0=1.0, uk=u, un=u, q_mode=Q_BZ, n_stab=nstab,
              precision=MIXED, seed=9, tile_cfg=1)
    g.init_fields(synth.fields(341, L, m.n_q)[None])
    g.sweep(2)
    phi = g.get_fields()[0]
    c = g.measure_tau()
    Bs = dqmc.propagators(m, phi)
    G00 = dqmc.green(m, phi, 0, Bs)
    for t in (0, 5, 10, 23, 40):
        want, _ = so5_correlator(*dqmc.green_displaced(m, phi, t, Bs), G00, n_phi)
        assert np.abs(c[0, t] - want).max() < 1e-10 * np.abs(want).max(), t
    g.close()


@pytest.mark.parametrize("n_phi,L,nstab,nch", [(36, 200, 10, 4), (100, 400, 8, 2)])
def test_tau_correlator_full_size_invariants(n_phi, L, nstab, nch):
    """At the N_phi = 36 and 100 shapes (paper cutoff, u = 1.5): carrying the
    three Green's functions through a block agrees with their recomputation
    from the stacks at the next boundary; antiperiodicity G(beta,0) = 1 - G(0),
    G(0,beta) = -G(0); C(L) = C(0); C(0) equals the equal-time S^i_{q=0}."""
    CFQMC = _gpu()
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.1, u0=1.0, uk=1.5, un=1.5, q_mode=Q_PAPER, n_stab=nstab,
              n_chains=nch, seed=17)
    g.init_fields()
    g.sweep(1)
    c, st = g.measure_tau(with_stab=True)
    assert np.isfinite(c).all()
    assert st.max() < 1e-8, st
    for k in range(nch):
        s, _ = g.observables(k)
        assert np.abs(c[k, 0].real - s).max() < 1e-9 * np.abs(s).max()
        assert rel(c[k, L], c[k, 0]) < 1e-8
    n = 2 * n_phi
    G0 = g.measure_G(0, 0)[:n, :n]
    gt0, g0t, _ = g.green_displaced(0, L)
    assert np.abs(gt0 - (np.eye(n) - G0)).max() < 1e-9
    assert np.abs(g0t + G0).max() < 1e-9
    g.close()


def test_tau_correlator_n100_against_the_oracle():
    """The N_phi = 100 shape of the main workload (paper cutoff, 933
    components, spin block 200: thirteen 16-wide tiles with a ragged tail) on
    a short imaginary-time axis the oracle evaluates directly: every tau
    within 1e-10."""
    CFQMC = _gpu()
    n_phi, L, nstab = 100, 12, 4
    m = Model(n_phi, L, 0.1, u0=1.0, uk=1.5, un=1.5, q_mode=Q_PAPER)
    phi = synth.fields(351, L, m.n_q)
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.1, u0=1.0, uk=1.5, un=1.5, q_mode=Q_PAPER, n_stab=nstab)
    g.init_fields(phi[None])
    c = g.measure_tau()
    Bs = dqmc.propagators(m, phi)
    G00 = dqmc.green(m, phi, 0, Bs)
    want = np.array([so5_correlator(*dqmc.green_displaced(m, phi, t, Bs), G00, n_phi)[0] for t in range(L + 1)])
    assert rel(c[0], want) < 1e-10, rel(c[0], want)
    g.close()
