"""GPU edge cases through the C ABI: the largest torus size of the paper
against the FP64 oracle, and the degenerate U = 0 point."""
import numpy as np
import pytest

import synth
from oracle import dqmc
from oracle.model import Model, Q_BZ, Q_PAPER

pytestmark = pytest.mark.gpu


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_03700_amd import CFQMC
    return CFQMC


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_largest_torus_n_phi_140_against_the_oracle():
    """N_phi = 140 (n = 280; paper cutoff, n_q = 1305), the largest torus of
    the paper, on a 16-slice axis the oracle evaluates directly: G(tau) at a
    block boundary, inside the axis and at beta, and ln w within 1e-10;
    Re tr G_4N = 2 N_phi."""
    CFQMC = _gpu()
    n_phi, L, nstab = 140, 16, 8
    m = Model(n_phi, L, 0.1, u0=1.0, uk=1.5, un=1.5, q_mode=Q_PAPER)
    phi = synth.fields(140, L, m.n_q)
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.1, u0=1.0, uk=1.5, un=1.5, q_mode=Q_PAPER, n_stab=nstab)
    assert g.n_q == m.n_q == 1305
    g.init_fields(phi[None])
    Bs = dqmc.propagators(m, phi)
    for tau in (0, nstab, L - 3, L):
        G = g.measure_G(0, tau)
        assert rel(G[:2 * n_phi, :2 * n_phi], dqmc.green(m, phi, tau, Bs)) < 1e-10, tau
        assert abs(np.trace(G).real - 2 * n_phi) < 1e-9
    ld, ldr = g.logdet(0), dqmc.logdet(m, phi, Bs)
    assert abs(ld.real - ldr.real) < 1e-10 * abs(ldr.real)
    g.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_u_zero_is_the_free_projected_band(precision):
    """U = 0: every channel coupling vanishes, each slice propagator is the
    identity (the projected band is flat), so G = 1/2 at every tau, ln w =
    2 n ln 2 (the oracle's closed form, pinned on the host), the
    recomputations agree exactly with the updates, and the weight stays
    sign-free while the fields move under the Gaussian action alone."""
    CFQMC = _gpu()
    n_phi, L, nch = 6, 16, 2
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.1, u0=0.0, uk=0.0, un=0.0, q_mode=Q_BZ, n_stab=4,
              precision=precision, n_chains=nch, chain_u=[(0.0, 0.0, 0.0)] * nch, seed=9)
    g.init_fields()
    phi0 = g.get_fields()
    st = g.sweep(2)
    half = 0.5 * np.eye(4 * n_phi)
    for k in range(nch):
        assert st[k]["max_stab_rel"] < 1e-12 and st[k]["max_phase_err"] < 1e-9
        assert 0 < st[k]["accepted"] <= st[k]["proposed"]
        for tau in (0, 5, L):
            assert np.abs(g.measure_G(k, tau) - half).max() < 1e-12
        ld = g.logdet(k)
        assert abs(ld.real - 2 * (2 * n_phi) * np.log(2.0)) < 1e-12 and abs(ld.imag) < 1e-12
    assert np.abs(g.get_fields() - phi0).max() > 0.0
    g.close()


def test_error_paths_leave_the_context_usable():
    """Calls before the fields exist report a state error, out-of-range
    chains, slices and sphere momenta report invalid arguments, and none of
    these changes the context: it then initialises, sweeps and measures as
    usual."""
    CFQMC = _gpu()
    from paper_2605_03700_amd import Q_SPHERE
    n_phi, L = 4, 8
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.1, q_mode=Q_BZ, n_stab=4, n_chains=2, seed=4)
    with pytest.raises(RuntimeError, match="ESTATE"):
        g.sweep(1)
    with pytest.raises(RuntimeError, match="ESTATE"):
        g.measure_G(0, 0)
    g.init_fields()
    with pytest.raises(RuntimeError, match="EINVAL"):
        g.measure_G(2, 0)
    with pytest.raises(RuntimeError, match="EINVAL"):
        g.measure_G(0, L + 1)
    st = g.sweep(1)
    assert all(s["max_stab_rel"] < 1e-10 for s in st)
    assert abs(np.trace(g.measure_G(1, L)).real - 2 * n_phi) < 1e-10
    g.close()
    s = CFQMC(n_phi=3, l_tau=4, dtau=0.02, uk=0.3, un=0.3, q_mode=Q_SPHERE, n_stab=2, exp_squarings=6)
    s.init_fields()
    with pytest.raises(RuntimeError, match="EINVAL"):
        s.structure_factors([(3, 0)])          # l = N_phi exceeds 2s = N_phi - 1
    with pytest.raises(RuntimeError, match="EINVAL"):
        s.structure_factors([(1, 2)])          # m > l
    assert np.isfinite(s.structure_factors([(1, 1)])).all()
    s.close()
