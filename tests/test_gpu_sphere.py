"""GPU parity of the spherical regularisation (Methods, "Spherical
regularization") against the FP64 oracle through the C ABI: G, ln w and the
observables at initialisation, replayed sweeps (FP64 and mixed), and the
imaginary-time correlator. Bars as on the torus: 1e-10 FP64, 1e-6 mixed.

The printed sphere density operators are O(1) per component (the torus ones
carry 1/(4 pi sqrt N)), so at equal coupling the slice exponents are one to
two orders larger: the cases use the sphere's small couplings (u ~ 0.2-0.5,
as in the paper's sphere runs), dtau = 0.02 (the paper's sphere benchmark
uses 0.01) and up to six scaling-and-squaring steps."""
import numpy as np
import pytest

import synth
from oracle import dqmc
from oracle.model import Model, Q_SPHERE
from oracle.observables import so5_correlator, so5_observables
from test_gpu_parity import _replay_compare

pytestmark = pytest.mark.gpu


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_03700_amd import CFQMC
    return CFQMC


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


DT = 0.02


@pytest.mark.parametrize("n_phi,L,nstab,u", [(1, 4, 3, 0.5), (2, 6, 3, 0.5), (3, 8, 4, 0.3), (4, 10, 4, 0.2),
                                             (6, 40, 5, 0.2), (12, 20, 4, 0.3)])
def test_sphere_green_logdet_observables_at_init(n_phi, L, nstab, u):
    CFQMC = _gpu()
    m = Model(n_phi, L, DT, u0=1.0, uk=u, un=u, q_mode=Q_SPHERE)
    assert m.n_q == n_phi * n_phi
    phi = synth.fields(500 + n_phi, L, m.n_q)
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=DT, u0=1.0, uk=u, un=u, q_mode=Q_SPHERE, n_stab=nstab, tile_cfg=1,
              exp_squarings=6)
    assert g.n_q == m.n_q
    g.init_fields(phi[None])
    Bs = dqmc.propagators(m, phi)
    n = 2 * n_phi
    for tau in sorted({0, 1, nstab, L - 1, L}):
        G = g.measure_G(0, tau)[:n, :n]
        assert rel(G, dqmc.green(m, phi, tau, Bs)) < 1e-10, tau
    ld, ldr = g.logdet(0), dqmc.logdet(m, phi, Bs)
    assert abs(ld.real - ldr.real) < 1e-10 * abs(ldr.real)
    s, m2 = g.observables(0)
    sr, m2r = so5_observables(dqmc.green(m, phi, L, Bs), n_phi, sphere=True)
    assert np.abs(s - sr.real).max() < 1e-10 * np.abs(sr).max()
    assert abs(m2 - m2r) < 1e-10 * abs(m2r)
    g.close()


def test_sphere_sweep_replay_parity_fp64():
    """N_phi = 6 on the sphere (36 components per channel), L = 40, n_stab = 4,
    two chains at u = 0.2 and 0.5, six sweeps of replayed noise: identical
    accept/reject sequences, fields, G and ln w within 1e-10."""
    CFQMC = _gpu()
    _replay_compare(CFQMC, 6, 40, 4, Q_SPHERE, None, [0.2, 0.5], 0, 6, 1e-10, dtau=DT, exp_squarings=6)


def test_sphere_sweep_replay_parity_single_orbital():
    """N_phi = 1 (s = 0: one orbital, the single l = 0 component), ragged block."""
    CFQMC = _gpu()
    _replay_compare(CFQMC, 1, 5, 2, Q_SPHERE, None, [0.3, 0.5], 0, 3, 1e-10, dtau=DT, exp_squarings=6)


def test_sphere_sweep_replay_parity_odd_orbitals():
    """N_phi = 5 (integer monopole strength s = 2), ragged last block."""
    CFQMC = _gpu()
    _replay_compare(CFQMC, 5, 11, 4, Q_SPHERE, None, [0.3], 0, 3, 1e-10, dtau=DT, exp_squarings=6)


def test_sphere_sweep_replay_parity_mixed():
    CFQMC = _gpu()
    st = _replay_compare(CFQMC, 6, 40, 4, Q_SPHERE, None, [0.2], 1, 2, 1e-6, dtau=DT, exp_squarings=6)
    assert st[0]["max_stab_rel"] < 1e-6


def test_sphere_tau_correlator_parity():
    CFQMC = _gpu()
    n_phi, L, nstab = 4, 12, 4
    m = Model(n_phi, L, DT, u0=1.0, uk=0.3, un=0.3, q_mode=Q_SPHERE)
    phi = synth.fields(540, L, m.n_q)
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=DT, u0=1.0, uk=0.3, un=0.3, q_mode=Q_SPHERE, n_stab=nstab, tile_cfg=1,
              exp_squarings=6)
    g.init_fields(phi[None])
    c = g.measure_tau()
    Bs = dqmc.propagators(m, phi)
    G00 = dqmc.green(m, phi, 0, Bs)
    want = np.array([so5_correlator(*dqmc.green_displaced(m, phi, t, Bs), G00, n_phi, sphere=True)[0]
                     for t in range(L + 1)])
    assert rel(c[0], want) < 1e-10
    g.close()


@pytest.mark.parametrize("n_phi,L", [(3, 8), (6, 20)])
def test_sphere_structure_factors_parity(n_phi, L):
    """S^i_{l,m} on the sphere (the correlation ratio uses l = 1) for chains on
    and off the SO(5) line against the oracle's Wick evaluation."""
    from oracle.model import gamma_matrices
    from oracle.observables import structure_factor
    CFQMC = _gpu()
    us = [(1.0, 0.3, 0.3), (1.0, 0.2, 0.5)]
    models = [Model(n_phi, L, DT, u0=a, uk=b, un=c, q_mode=Q_SPHERE) for (a, b, c) in us]
    phi = np.stack([synth.fields(560 + 3 * k + n_phi, L, models[0].n_q) for k in range(len(us))])
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=DT, q_mode=Q_SPHERE, n_stab=4, n_chains=len(us), chain_u=us, tile_cfg=1,
              exp_squarings=6)
    g.init_fields(phi)
    qs = [(0, 0), (1, 0), (1, 1), (2, 1), (n_phi - 1, n_phi - 1), (n_phi - 1, 0)]
    s = g.structure_factors(qs)
    for k in range(len(us)):
        G = dqmc.green(models[k], phi[k], 0)
        want = np.array([[structure_factor(G, n_phi, gm, l, m, sphere=True) for gm in gamma_matrices()]
                         for (l, m) in qs])
        assert rel(s[k], want) < 1e-10, (k, rel(s[k], want))
        s0, _ = g.observables(k)
        assert np.abs(s[k, 0].real - s0).max() < 1e-10 * np.abs(s0).max()
    with pytest.raises(RuntimeError):
        g.structure_factors([(1, 2)])            # m > l
    g.close()


def test_sphere_n59_at_init_against_the_oracle():
    """The paper's largest sphere, N_phi = 59 (3481 components per channel,
    spin block 118), on a short imaginary-time axis: G(tau), ln w and
    S^i_{l,m} at l = 0, 1 within 1e-10 of the oracle."""
    from oracle.model import gamma_matrices
    from oracle.observables import structure_factor
    CFQMC = _gpu()
    n_phi, L, nstab = 59, 6, 3
    m = Model(n_phi, L, 0.01, u0=1.0, uk=0.2, un=0.2, q_mode=Q_SPHERE)
    phi = synth.fields(590, L, m.n_q)
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.01, u0=1.0, uk=0.2, un=0.2, q_mode=Q_SPHERE, n_stab=nstab,
              exp_squarings=10)
    g.init_fields(phi[None])
    Bs = dqmc.propagators(m, phi)
    n = 2 * n_phi
    for tau in (0, 2, nstab, L):
        assert rel(g.measure_G(0, tau)[:n, :n], dqmc.green(m, phi, tau, Bs)) < 1e-10, tau
    ld, ldr = g.logdet(0), dqmc.logdet(m, phi, Bs)
    assert abs(ld.real - ldr.real) < 1e-10 * abs(ldr.real)
    G = dqmc.green(m, phi, 0, Bs)
    qs = [(0, 0), (1, 0), (1, 1)]
    s = g.structure_factors(qs)
    want = np.array([[structure_factor(G, n_phi, gm, l, mm, sphere=True) for gm in gamma_matrices()]
                     for (l, mm) in qs])
    assert rel(s[0], want) < 1e-10
    g.close()
